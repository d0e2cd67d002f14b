/*
 * vfpi.h -- C ABI of the V-FPI contact solver for AMD Instinct MI355X (gfx950).
 *
 * Method: "Large-Dimensional Multibody Dynamics Simulation Using Contact
 * Nodalization and Diagonalization" (J. Lee, M. Lee, D. Lee).  One time step
 * solves the linear contact problem
 *
 *     A v = b + J_c^T lambda,  Signorini-Coulomb complementarity per contact
 *                                              (Sec. II, eq. lindyn, eq. scc)
 *
 * with the velocity fixed-point iteration (V-FPI, Alg. 1): each sweep is
 *     v*      = v^l - W (A v^l - b)                           (eq. pgd1)
 *     eta_m   = R_m v*_i                                      (eq. subp, nodal J_c)
 *     lambda_m = ProjectFC(-(eta_m + phi_m e1) / gamma_m)     (Alg. 2, eq. operator)
 *     v^{l+1} = v* + W J_c^T lambda                           (eq. vup)
 *     theta   = ||v^{l+1} - v^l||_2,  stop if theta < tol or l = max_iters
 * where W is diagonal with one shared value w_i on the three DOFs of every
 * contact node, so that J_c W J_c^T = diag(gamma_m I3) with gamma_m = w_i
 * (Prop. 3, eq. diagonal).
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers owned by the caller, except the
 *    descriptor structs themselves (host memory, read during the call only).
 *  - Work is enqueued asynchronously on `stream`; results (outputs and the
 *    device-side stats record) are valid once the stream has synchronized.
 *  - Inputs are never modified.  `v` is in/out (warm start in, solution out);
 *    every other output is fully overwritten.
 *  - Sizes: N nodes, n = 3N DOFs, node-major vectors (x,y,z of node 0, ...).
 *    Indices are int32.
 *  - Synchronous argument errors return a negative VFPI_E_* code and enqueue
 *    nothing.  Data errors that need the device to detect are reported in
 *    stats->status (VFPI_S_* bits); when any is set the solve is skipped:
 *    v is left as given, lambda is zeroed, iters = 0.
 *  - A context owns device workspace sized at creation; one context must not
 *    be used by two streams at once (calls on one stream are ordered).
 */
#ifndef VFPI_H
#define VFPI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes (synchronous) ---------------------------------------- */
#define VFPI_OK              0
#define VFPI_E_NULL         -1  /* a required pointer is NULL                  */
#define VFPI_E_SHAPE        -2  /* inconsistent sizes (negative, n_c > N, ...)  */
#define VFPI_E_OPTS         -3  /* invalid option value                         */
#define VFPI_E_CAPACITY     -4  /* larger than the context was created for     */
#define VFPI_E_UNSUPPORTED  -5  /* valid input the library does not solve      */
#define VFPI_E_HIP          -6  /* a HIP runtime call failed                    */
#define VFPI_E_NO_TAPE      -7  /* backward without a forward tape              */

/* ---- device status (stats.status) -------------------------------------- */
#define VFPI_S_CONVERGED        0x000  /* theta < tol at the break            */
#define VFPI_S_MAXITER          0x001  /* stopped at max_iters (or fixed_iters) */
#define VFPI_S_NONFINITE        0x010  /* NaN/Inf in A, b, v, R, phi or mu     */
#define VFPI_S_NOT_NODAL        0x020  /* J_c row is neither [R] nor [R, -R]      */
#define VFPI_S_NOT_ORTHONORMAL  0x040  /* max |R R^T - I| > 1e-10 (1e-5 in FP32) */
#define VFPI_S_SHARED_NODE      0x080  /* a node carries two contacts (Prop. 3)  */
#define VFPI_S_NONPOS_DIAG      0x100  /* a_ii <= 0 or no diagonal block        */
#define VFPI_S_BAD_PATTERN      0x200  /* column index out of range / out of env */
#define VFPI_S_BAD_W            0x400  /* user W not positive, or unequal on a contact node */
#define VFPI_S_BAD_MU           0x800  /* mu < 0                               */
#define VFPI_S_SYNC_TIMEOUT    0x1000  /* a workgroup of the persistent kernel waited
                                          for another for seconds and gave up; the
                                          results are not valid (not expected to
                                          happen: a guard against a hang) */

/* ---- step-size matrix W (Sec. IV-C) ------------------------------------ */
#define VFPI_W_FROBENIUS    0  /* w_d = a_dd/||A_d*||^2, shared on contact nodes (Sec. IV-C.1) */
#define VFPI_W_USER_DIAG    1  /* opts.w_user[n], equal on the 3 DOFs of each contact node */
#define VFPI_W_USER_SCALAR  2  /* W = opts.alpha_user I                        */
#define VFPI_W_BB1          3  /* Barzilai-Borwein s's/s'z (Sec. IV-C.2)       */
#define VFPI_W_BB2          4  /* Barzilai-Borwein s'z/z'z (Sec. IV-C.2)       */
/* BB modes: W = alpha^l I with alpha^1 = 1/max_d sum_j |a_dj| and, for l >= 2,
 * s = v^l - v^{l-1}, z = A v^l - A v^{l-1}; alpha is kept when the quotient is
 * not positive.  vfpi_step only, launch kinds 1 and 3, no Chebyshev
 * (VFPI_E_UNSUPPORTED otherwise); two grid reductions per sweep.  The tape
 * of a BB step holds W = alpha I of the last sweep; the adjoint iteration of
 * vfpi_step_backward contracts only if that alpha is below 2 / lambda_max(A),
 * which a long BB step need not be (differentiate a FROBENIUS step instead). */

/* ---- ProjectFC (eq. operator) ------------------------------------------ */
#define VFPI_PROJ_STRICT    0  /* normal clamp + disk projection (default)     */
#define VFPI_PROJ_PROXIMAL  1  /* Euclidean projection onto the friction cone  */

/* Block-sparse row matrix with 3x3 blocks (the system matrix A_k, eq. akbk).
 * row_ptr[n_nodes+1], col_idx[nnzb] (node indices), val[9*nnzb] row-major
 * blocks, double (vfpi_step, vfpi_step_backward) or float (vfpi_step_batched).
 * A must be symmetric positive definite with a diagonal block in every row;
 * symmetry is the caller's promise (it is not checked). */
typedef struct {
  int32_t n_nodes;
  int32_t nnzb;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
} vfpi_bsr;

/* Nodal contact Jacobian J_c (eq. jcnode) in the same block-row form, one
 * block row per contact: an S-contact (node against the static environment)
 * is one block R_m in SO(3) (row 0 = contact normal, rows 1-2 = tangents) at
 * the contact's node i; a D-contact (node against node) is R_m at node i
 * followed by -R_m (bitwise the negation) at node j != i, the relative
 * velocity R_m (v_i - v_j) having its normal along row 0.  phi[n_contacts] is
 * the normal offset term and mu[n_contacts] >= 0 the friction coefficient
 * (eq. scc).  At most one contact per node (either node of a D-contact
 * counts).  Element type as for vfpi_bsr.val. */
typedef struct {
  int32_t n_contacts;
  int32_t nnzb;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  const void* phi;
  const void* mu;
  const void* mu2;   /* NULL: isotropic friction.  Else [n_contacts] >= 0: anisotropic
                        friction on the elliptic cone lambda_n^2 >= t1^2/mu^2 + t2^2/mu2^2
                        (tangents = rows 1, 2 of R; Sec. III-E), solved by the strict
                        operator, which gives the maximal-dissipation impulse (Prop. 6).
                        Not with VFPI_PROJ_PROXIMAL (VFPI_E_UNSUPPORTED). */
} vfpi_contacts;

typedef struct {
  int32_t max_iters;     /* l_max of Alg. 1 (>= 0)                             */
  int32_t fixed_iters;   /* 1: ignore tol, run exactly max_iters sweeps         */
  double  tol;           /* theta_th of Alg. 1, absolute (m/s)                  */
  int32_t w_mode;        /* VFPI_W_*                                            */
  int32_t projection;    /* VFPI_PROJ_*                                         */
  const void* w_user;    /* device [n], VFPI_W_USER_DIAG only                   */
  double  alpha_user;    /* VFPI_W_USER_SCALAR only                             */
  int32_t reuse_w;       /* 1: keep the row sums a_dd, ||A_d*||^2 of the previous
                            call on this context (W reuse across steps, Sec. IV-C) */
  int32_t variant;       /* launch variant: kind | chunk slots << 8 | workgroup cap << 16
                            | LDS levels << 24 | load group << 26 | sync << 28.
                            vfpi_step kinds: 1 grid, lane per node; 2 grid, lane per row;
                            3, 4 the same in one workgroup; 5 grid, the node's first
                            block levels of A in registers and the next ones in LDS
                            (LDS levels: 0 when rows average more than 9 blocks, 1 off,
                            2 on; refused with VFPI_E_OPTS when the grid needs more
                            than one workgroup per CU; without Chebyshev and BB step
                            sizes it takes the stop test of sweep l after
                            sweep l + 1 and synchronizes a workgroup only with the
                            workgroups owning its rows' columns, unless sync = 1, which
                            keeps a full grid reduction after every sweep; the results
                            are the same).  Load group (kind 1 with 8
                            chunk slots): levels of A loaded together, 1 two, else
                            four.  0 = library
                            default: kind 5 with the fewest chunk slots (2, 4, 5, 6, 8)
                            that fit, else kind 1 with 8 slots and groups of two
                            levels (also with BB step sizes, which take 4 slots).
                            vfpi_step_backward: 0 or 5 register-resident (S- and
                            D-contacts), 1 streaming, 3 one workgroup.  Batched
                            kinds: see below. */
  int32_t cheby_ls;      /* 0: off; l_s >= 1: Chebyshev acceleration (Alg. 3):
                            nu = 1 before sweep l_s, 2/(2 - rho^2) at l_s, then
                            4/(4 - rho^2 nu); rho = min(theta_l / theta_{l-1}, 1) */
  double  cheby_u;       /* under-relaxation u of the accelerated update (0 < u <= 1;
                            0 is read as 1):
                            v^{l+1} = nu (u (v** - v^l) + v^l - v^{l-1}) + v^{l-1} */
  double  omega;         /* invertible contact (Sec. III-E, eq. invt): Omega_c = omega I,
                            the contact step uses gamma_m + omega (omega >= 0; 0 = off).
                            vfpi_step_backward must get the forward call's value. */
} vfpi_opts;

/* Written on the device; `stats` points to device memory. */
typedef struct {
  int32_t iters;         /* sweeps executed (l at the break)                   */
  int32_t status;        /* VFPI_S_*                                           */
  double  theta;         /* residual of the last sweep (+inf if none ran)      */
  int32_t n_open, n_stick, n_slip;  /* branch counts of the last sweep        */
  int32_t reserved;
} vfpi_stats;

/* Create a context able to solve problems up to the given sizes.
 * max_envs bounds vfpi_step_batched (0 if unused).  Allocates device memory
 * on the current device.  Returns VFPI_E_SHAPE for negative sizes,
 * VFPI_E_HIP if allocation fails (then *ctx is NULL). */
typedef struct vfpi_ctx vfpi_ctx;
int vfpi_create(vfpi_ctx** ctx, int32_t max_nodes, int32_t max_nnzb, int32_t max_contacts,
                int32_t max_envs);
/* Free a context (NULL is a no-op).  Synchronizes the device first. */
int vfpi_destroy(vfpi_ctx* ctx);

/* Bytes of the forward tape needed by vfpi_step_backward (w, v, lambda*,
 * branch per contact).  Host-only arithmetic, no device access. */
int64_t vfpi_tape_bytes(int32_t n_nodes, int32_t n_contacts);

/* One plain FP64 V-FPI solve (Alg. 1 inner loop, Alg. 2 contact step).
 *   A       FP64 system matrix A_k (eq. lindyn)
 *   b       [n]  right-hand side b_k
 *   Jc      FP64 nodal contact Jacobian (S- and D-contacts), phi, mu, mu2
 *   v       [n]  in: warm start v^1 (Sec. V-A.5); out: v^{l+1} of the last sweep
 *   lambda  [3 n_c] out: contact impulses (n, t1, t2) of the last sweep
 *   opts    options (host struct)
 *   stats   device vfpi_stats, written at the end
 *   tape    NULL, or a device buffer of vfpi_tape_bytes(N, n_c) bytes that
 *           receives what vfpi_step_backward needs
 * Errors: VFPI_E_NULL, VFPI_E_SHAPE (also Jc->nnzb > 2 n_c), VFPI_E_OPTS,
 * VFPI_E_CAPACITY, VFPI_E_UNSUPPORTED (BB modes with Chebyshev or with launch
 * kinds other than 1, 3 and 5; mu2 with VFPI_PROJ_PROXIMAL), VFPI_E_HIP. */
int vfpi_step(vfpi_ctx* ctx, const vfpi_bsr* A, const double* b, const vfpi_contacts* Jc,
              double* v, double* lambda, const vfpi_opts* opts, vfpi_stats* stats,
              void* tape, hipStream_t stream);

/* Many independent problems ("environments") in one launch, FP32 arithmetic
 * with the residual theta accumulated and tested in FP64.  The envs are
 * concatenated block-diagonally: env e owns nodes
 * [env_node_off[e], env_node_off[e+1]) and contacts [env_con_off[e],
 * env_con_off[e+1]); A, b, Jc, v, lambda use global node/contact indices and
 * FP32 values.  env_order (device [n_env] permutation, or NULL) is the order
 * in which the persistent kernel's work queue hands out envs (largest first is
 * a good choice).  Launch kinds (opts.variant): 1 lane per node, 2 lane per
 * row, 3 lane per node with two workgroups per CU, 4 lane per node with the
 * environment's iterate in LDS: 8 waves per workgroup (the first 512 nodes
 * keep their first 9 block levels of A in registers for the whole step, the
 * rest stream A two levels at a time, four with load group 1 << 26) or 16
 * waves (all of A streamed); environments of up to 3,072 nodes, larger ones
 * run kind 1's loop in the same launch; 0 = kind 4 with 8 waves.
 * per_env_stats: device [n_env].  Every option applies to
 * every env; each env stops on its own theta.  W modes: FROBENIUS,
 * USER_SCALAR.  Errors as vfpi_step. */
int vfpi_step_batched(vfpi_ctx* ctx, int32_t n_env, const int32_t* env_node_off,
                      const int32_t* env_con_off, const int32_t* env_order,
                      const vfpi_bsr* A, const float* b, const vfpi_contacts* Jc,
                      float* v, float* lambda, const vfpi_opts* opts,
                      vfpi_stats* per_env_stats, hipStream_t stream);

/* Adjoint of a converged vfpi_step (implicit differentiation through the
 * fixed point, with the projection's active branch per contact):
 * given dL/dv and optionally dL/dlambda of the step's outputs, writes dL/db,
 * dL/dA (on A's pattern, NULL to skip), dL/dphi, dL/dmu and (anisotropic
 * friction) dL/dmu2.
 *   A, Jc     the same matrices as the forward call (FP64), Jc->mu2 included
 *   tape      the buffer filled by the forward call
 *   grad_v    [n];  grad_lambda [3 n_c] or NULL (zero)
 *   grad_b    [n] out; grad_A_val [9 nnzb] out or NULL; grad_phi, grad_mu [n_c] out
 *   grad_mu2  [n_c] out when Jc->mu2 != NULL (required then), else ignored.
 *             The slip branch on the elliptic cone is differentiated
 *             implicitly through the ellipse's closest-point condition; with
 *             one coefficient zero (a segment) the derivative in that
 *             coefficient is one-sided (mu >= 0).
 *   opts      max_iters / tol of the adjoint's own fixed-point iteration
 * The adjoint u solves u = g + (I - A W) G^T u with G = I - W J^T D_P Gamma^-1 J
 * (D_P = projection Jacobian of the last sweep), by transposed sweeps that
 * reuse the forward's layout; D-contacts, opts.omega and opts.projection
 * (both of which must equal the forward's) are supported.  Errors as
 * vfpi_step, plus VFPI_E_NO_TAPE for tape == NULL and VFPI_E_UNSUPPORTED for
 * mu2 with VFPI_PROJ_PROXIMAL (as in the forward). */
int vfpi_step_backward(vfpi_ctx* ctx, const vfpi_bsr* A, const vfpi_contacts* Jc,
                       const void* tape, const double* grad_v, const double* grad_lambda,
                       double* grad_b, double* grad_A_val, double* grad_phi, double* grad_mu,
                       double* grad_mu2, const vfpi_opts* opts, vfpi_stats* stats,
                       hipStream_t stream);

/* ---- the plain solve without allocation --------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * vfpi_step_noalloc runs exactly vfpi_step's kernels (same results, bit for
 * bit, for the same inputs and options) but needs no context: its workspace
 * lies in one device array of VFPI_NOALLOC_SCRATCH_BYTES inside the library,
 * one copy per GPU, held from the first call on that GPU until the process
 * ends.  The call allocates and frees nothing.  The caller still passes every
 * input and output (device pointers, as for vfpi_step); the workspace takes
 *   84 nnzb + 316 N + 112 n_c + 1,671,680 bytes
 * (each of its 14 parts rounded up to 256 bytes), which must fit the array:
 * about 26,900 nodes of a cloth with 9 blocks per row and a contact on every
 * node (about 29,700 without contacts).  Every call on one GPU
 * shares that GPU's array, and each call starts by clearing the parts that
 * must start at zero; two calls that overlap on one GPU (on different
 * streams, or from different threads) race and give undefined results.
 * Calls must be ordered, e.g. on one stream.  The workspace is used on the
 * current device.  opts->reuse_w is refused (another call may have
 * overwritten the row sums).  The timing aid does not apply.
 * Errors: as vfpi_step; VFPI_E_CAPACITY when the workspace does not fit;
 * VFPI_E_OPTS for reuse_w. */
#define VFPI_NOALLOC_SCRATCH_BYTES (32u << 20)
int vfpi_step_noalloc(const vfpi_bsr* A, const double* b, const vfpi_contacts* Jc, double* v,
                      double* lambda, const vfpi_opts* opts, vfpi_stats* stats, void* tape,
                      hipStream_t stream);

/* ---- virtual nodes (Sec. III-A, eq. vforce, eq. vnode) ------------------
 * A contact at a point that is not a node (a point of a triangle, of a rigid
 * body) gets a temporary virtual node q tied to the point's velocity J_v v_o
 * by the viscous force -k_v (J_v v_o - v_q).  The solver then runs on
 *   A = [A_o + k_v J_v^T J_v, -k_v J_v^T; -k_v J_v, k_v I],  b = [b_o; 0]
 * (SPD, Prop. 1), whose solution approaches the original contact problem as
 * k_v grows (Prop. 2).  Virtual node q is node n_o + q of the result; contacts
 * on it are ordinary S- or D-contacts in that numbering.
 * J_v: n_v block rows (jv_ptr[n_v+1], jv_col = original node of each 3x3
 * block, jv_val[9 nnz] row-major), distinct columns within a row.  A_o's rows
 * must have sorted column indices.
 *
 * vfpi_vnode_pattern (host arrays, no device access): block pattern of A,
 * rows sorted by column, the virtual columns last in each original row.
 * With aug_col_idx == NULL only aug_row_ptr[n_o+n_v+1] and *aug_nnzb are
 * written (size query).  Errors: VFPI_E_NULL, VFPI_E_SHAPE (an index out of
 * range, decreasing offsets, a repeated column in a J_v row),
 * VFPI_E_CAPACITY (more than cap blocks). */
int vfpi_vnode_pattern(int32_t n_o, const int32_t* row_ptr, const int32_t* col_idx, int32_t n_v,
                       const int32_t* jv_ptr, const int32_t* jv_col, int32_t* aug_row_ptr,
                       int32_t* aug_col_idx, int64_t cap, int64_t* aug_nnzb);

/* vfpi_vnode_values (device arrays, FP64, asynchronous on `stream`): the
 * block values of A on the pattern from vfpi_vnode_pattern (copied to the
 * device), b = [b_o; 0] and the warm start v = [v_o; J_v v_o].
 * Errors: VFPI_E_NULL, VFPI_E_SHAPE, VFPI_E_OPTS (k_v not positive and
 * finite), VFPI_E_HIP. */
int vfpi_vnode_values(const vfpi_bsr* A_o, const double* b_o, const double* v_o, int32_t n_v,
                      const int32_t* jv_ptr, const int32_t* jv_col, const double* jv_val, double k_v,
                      const int32_t* aug_row_ptr, const int32_t* aug_col_idx, double* aug_val,
                      double* b, double* v, hipStream_t stream);

/* Profiling aid.  While enabled on a context, vfpi_step, vfpi_step_batched
 * and vfpi_step_backward record HIP events on their stream before the setup
 * kernels, between setup and the solve kernel, and after the solve kernel
 * (do not enable it for calls captured into a graph).  vfpi_timing_read
 * waits for the last call's events and returns the two durations in
 * milliseconds.  Errors: VFPI_E_NULL, VFPI_E_OPTS (read without an enabled,
 * recorded call), VFPI_E_HIP. */
int vfpi_timing_enable(vfpi_ctx* ctx, int32_t on);
int vfpi_timing_read(vfpi_ctx* ctx, float* setup_ms, float* solve_ms);

/* Static description of a return code. */
const char* vfpi_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* VFPI_H */
