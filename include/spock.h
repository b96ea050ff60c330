/*
 * spock.h - C ABI of the MI355X (gfx950) implementation of SPOCK, the
 * SuperMann-accelerated Chambolle-Pock method for multistage risk-averse
 * optimal control on a scenario tree (Bodard, Moran, Schuurmans, Patrinos,
 * Sopasakis, arXiv 2212.01110).
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status: SPOCK_OK (0) or a negative error
 *    code. On error no output buffer and no handle is modified.
 *  - Host arrays (plain C pointers) are read during the call and copied; the
 *    caller keeps ownership. Device pointers (suffix _dev) are caller-owned
 *    HIP device allocations; they are read/written only on the given stream,
 *    and the call returns once that work is enqueued, except where a function
 *    says it synchronises.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Precision: a problem is factored in FP64 on the host, then its bulk data
 *    is stored in SPOCK_FP64 or SPOCK_FP32. Device vectors of that problem
 *    (z, eta, v) use that element type; x0 is always FP64.
 *  - Handles are not thread safe; one handle is used by one stream at a time.
 *
 * Vector layout (section 5.2, "Operator splitting"): nodes in breadth-first
 * order with contiguous children (Fig. 1), all leaves at stage N.
 *   z   = (s^0,
 *          x^i for every node            [num_nodes][nx],
 *          u^i for every nonleaf node    [num_nonleaf][nu],
 *          per nonleaf i: y^i (2 n_i + 1), tau^c for c in ch(i), s^c for c in ch(i))
 *   eta = (per nonleaf i: y^i (2 n_i + 1), s^i - b^i'y^i, x^i (nx), u^i (nu);
 *          per non-root c: Q_c^{1/2} x^{anc c} (nx), R_c^{1/2} u^{anc c} (nu), tau^c/2, tau^c/2;
 *          per leaf j: x^j (nx), Q_N^{1/2} x^j (nx), s^j/2, s^j/2)
 *   v   = (z, eta), n_v = n_z + n_eta; n_i = |ch(i)|, b^i = (p^{ch(i)}, 0, 1)
 *   with p^c = pi^c / pi^{anc c} (conditional probability) and y^i the AV@R
 *   conic dual variable (section 4.3: E = [aI, -I, 1]', K = R^{2n}_+ x {0}).
 */
#ifndef SPOCK_H
#define SPOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spock_tree spock_tree;        /* opaque, library-owned */
typedef struct spock_problem spock_problem;  /* opaque, library-owned */

enum {
  SPOCK_OK = 0,
  SPOCK_EINVAL = -1,      /* null pointer, bad size, bad setting, x0 precision */
  SPOCK_ETREE = -2,       /* not breadth-first / children not contiguous / leaf not at stage N */
  SPOCK_EPROB = -3,       /* pi <= 0, non-finite, children not summing to their parent */
  SPOCK_EBOX = -4,        /* lower bound above upper bound, or x0 outside the root box */
  SPOCK_EFACTOR = -5,     /* Alg. 1 hit a non-SPD R~ or a non-finite value */
  SPOCK_EHIP = -6,        /* a HIP runtime call failed */
  SPOCK_ENOMEM = -7,      /* host or device allocation failed */
  SPOCK_EUNSUPPORTED = -8, /* nx or nu above 64, or an unsupported mode */
  SPOCK_ETOOBIG = -9       /* the problem needs more than the fixed scratch of spock_T_noalloc */
};

/* spock_info.status: outcome of an iteration, not an error. SPOCK_REJECTED is
 * reported by spock_solve_batched for an instance whose x0 lies outside its
 * root box (that instance is skipped, its v_io left untouched). */
enum { SPOCK_CONVERGED = 0, SPOCK_MAXITER = 1, SPOCK_NUMERICAL = 2, SPOCK_REJECTED = 3 };
enum { SPOCK_FP64 = 0, SPOCK_FP32 = 1 };
enum { SPOCK_METHOD_CP = 0, SPOCK_METHOD_SPOCK = 1 };
/* How the Anderson least squares (section 6.2) is solved: AUTO takes the
 * device Gram solve for m <= 4 and the QR-updated form above; GRAM: normal
 * equations with an FP64 Cholesky on the device (m <= 4); QR: a thin QR
 * factorisation updated at every push (Gram-Schmidt with reorthogonalisation
 * for a new column, Givens rotations to drop the oldest; m <= 10). */
enum { SPOCK_AA_AUTO = 0, SPOCK_AA_GRAM = 1, SPOCK_AA_QR = 2 };

/* Scenario tree (section 4.1). anc[num_nodes] with anc[0] = -1 and
 * 0 <= anc[i] < i, nondecreasing in i (breadth-first, contiguous children);
 * prob[num_nodes] node probabilities pi^i > 0 with every node's children
 * summing to it (relative tolerance 1e-10) and pi^0 = 1. Every leaf must sit at
 * the last stage N >= 1. Errors: SPOCK_EINVAL (null/num_nodes < 2),
 * SPOCK_ETREE, SPOCK_EPROB, SPOCK_ENOMEM. */
int spock_tree_create(int32_t num_nodes, const int32_t* anc, const double* prob,
                      spock_tree** out);
int spock_tree_destroy(spock_tree* tree);
/* horizon N, nonleaf count and leaf count of a tree */
int spock_tree_shape(const spock_tree* tree, int32_t* N, int32_t* num_nonleaf,
                     int32_t* num_leaves);

/* Problem data (section 4.1, "Dynamics", "Constraints", "Quadratic costs";
 * section 4.2 for AV@R). Host arrays, row-major, indexed by node; row 0 of
 * per-edge data (A, B, q, r) is unused. Q, R and Q_N are diagonal and given by
 * their diagonals unless the dense matrices below are given; the constraint
 * sets are boxes (Gamma = identity) unless polyhedral rows are given.
 *   A  [num_nodes][nx][nx], B [num_nodes][nx][nu]: x^c = A^c x^{anc c} + B^c u^{anc c}
 *   q  [num_nodes][nx] > 0, r [num_nodes][nu] > 0: stage cost x'Q^c x + u'R^c u charged at c
 *   qN [num_nodes][nx] >= 0: terminal cost x'Q_N x, read at leaves
 *   xmin, xmax [num_nodes][nx]: state box of every node (root included)
 *   umin, umax [num_nodes][nu]: input box, read at nonleaf nodes
 *   a_risk [num_nodes]: AV@R parameter a in [0, 1] of each nonleaf node
 *   precision: SPOCK_FP64 or SPOCK_FP32 storage of the iteration data
 *   alpha: CP step size; <= 0 selects 0.99 / ||L||; otherwise must satisfy
 *          0 < alpha ||L|| < 1 (section 3). */
/* General coherent risk measures in the conic form of section 4.3: at
 * nonleaf node i, rho(Z) = max { mu'Z : E^i mu + F^i nu <=_K b^i } with
 * K = R^{kpos_i}_+ x {0}^{ny_i - kpos_i} (the first kpos_i rows are
 * inequalities, the rest equalities); the problem then carries the conic
 * dual y^i (ny_i entries) in place of AV@R's 2 n_i + 1, and S2 becomes the
 * kernel of [E' -I -I; F' 0 0]. Per nonleaf node i in breadth-first order,
 * concatenated (leaves have none):
 *   ny[num_nodes], nnu[num_nodes], kpos[num_nodes] (0 at leaves; ny_i >= 1,
 *   0 <= kpos_i <= ny_i, nnu_i >= 0)
 *   E: [ny_i][n_i] row-major, F: [ny_i][nnu_i] (NULL if every nnu_i is 0),
 *   b: [ny_i]. */
typedef struct {
  const int32_t *ny, *nnu, *kpos;
  const double *E, *F, *b;
} spock_risk_data;

/* General polyhedral constraints (section 4.1, eq. constraints): at nonleaf
 * node i, cmin <= Gamma_x x^i + Gamma_u u^i <= cmax (nc rows); at leaf j,
 * cNmin <= Gamma_N x^j <= cNmax (ncN rows). Row-major per node:
 * Gx [num_nodes][nc][nx], Gu [num_nodes][nc][nu], cmin, cmax [num_nodes][nc]
 * (read at nonleaf nodes); GN [num_nodes][ncN][nx], cNmin, cNmax
 * [num_nodes][ncN] (read at leaves). Bounds may be +-infinity, nc, ncN >= 1. */
typedef struct {
  int32_t nc, ncN;
  const double *Gx, *Gu, *cmin, *cmax;
  const double *GN, *cNmin, *cNmax;
} spock_constraint_data;

typedef struct {
  int32_t nx, nu;
  const double *A, *B;
  const double *q, *r, *qN;
  const double *xmin, *xmax, *umin, *umax;
  const double* a_risk;
  int32_t precision;
  double alpha;
  /* NULL: AV@R_a of a_risk at every nonleaf node. Otherwise the general
   * conic risk above (a_risk is not read). */
  const spock_risk_data* risk;
  /* NULL: the boxes xmin..umax. Otherwise the polyhedral constraints above
   * (the boxes are not read, and x0 is not checked against a root box). */
  const spock_constraint_data* cons;
  /* NULL: the diagonals q, r, qN. Otherwise dense symmetric cost matrices
   * (section 4.1), all three: Qm [num_nodes][nx][nx] (row c: Q^c, positive
   * semidefinite), Rm [num_nodes][nu][nu] (positive definite) and QNm
   * [num_nodes][nx][nx] (positive semidefinite, read at leaves); q, r, qN are
   * then not read (may be NULL). The cost rows of L carry their symmetric
   * square roots. A problem with dense costs runs the general kernels.
   * Errors: SPOCK_EINVAL when only some are given, or a matrix is not finite,
   * not symmetric (1e-12 relative) or not (semi)definite as stated; the
   * batched engines and spock_backward return SPOCK_EUNSUPPORTED for it. */
  const double *Qm, *Rm, *QNm;
} spock_problem_data;

/* Runs Alg. 1 (offline S1 factorisation) in FP64 on the host, computes ||L||
 * from its block-diagonal structure (remark after the definition of L) and
 * uploads the stage-ordered device layout. Synchronises. The tree must
 * outlive the problem. With general risk or constraint data the vector
 * layout follows it (y^i of ny_i entries; nc constraint rows in place of
 * (x^i, u^i) in group 1 of eta, ncN in place of x^j in group 3), and the
 * problem runs in spock_solve, the operator entry points and
 * spock_T_noalloc; spock_solve_batched and spock_backward reject it with
 * SPOCK_EUNSUPPORTED, and spock_info.V_nested is NaN for it. Errors:
 * SPOCK_EINVAL, SPOCK_EBOX, SPOCK_EFACTOR, SPOCK_EUNSUPPORTED, SPOCK_EHIP,
 * SPOCK_ENOMEM. */
int spock_problem_factor(const spock_tree* tree, const spock_problem_data* data,
                         spock_problem** out);
int spock_problem_destroy(spock_problem* prob);
/* sizes and step: n_z, n_eta, alpha and ||L|| (any pointer may be NULL) */
int spock_problem_sizes(const spock_problem* prob, int64_t* n_z, int64_t* n_eta,
                        double* alpha, double* norm_L);
/* The family-to-lane mapping the next evaluation of T will use (as
 * spock_info.mapping), the workgroups of the dataflow launch (0 for the
 * other mappings) and whether the dataflow form has been given up for this
 * problem (1) after one of its bounded waits gave up. Any pointer may be
 * NULL. Errors: SPOCK_EINVAL. */
int spock_problem_mapping(const spock_problem* prob, int32_t* mapping, int32_t* flow_grid,
                          int32_t* flow_failed);

/* Solver settings (section 3 termination; Alg. 3 parameters). method CP runs
 * v <- T(v); method SPOCK runs Alg. 3 with Anderson memory m (1..10; 1..4
 * with anderson = SPOCK_AA_GRAM and in spock_solve_batched).
 * Parameters follow Alg. 3: c0, c1, c2 in [0,1), beta, sigma in (0,1),
 * lambda in (0,2); max_ls caps the backtracking (then a plain KM step is
 * taken). compute_nested != 0 also evaluates the exact nested AV@R cost of the
 * returned trajectory on the host (one device-to-host copy). */
typedef struct {
  double eps_abs, eps_rel;
  int32_t max_iters, method, m, max_ls;
  double c0, c1, c2, beta, sigma, lambda;
  int32_t compute_nested;
  int32_t anderson;        /* SPOCK_AA_AUTO, SPOCK_AA_GRAM or SPOCK_AA_QR */
} spock_settings;

/* Fills the defaults: eps 1e-4/1e-4, max_iters 20000, SPOCK, m = 3,
 * max_ls = 20, c0 = c1 = c2 = 0.99, beta = 0.5, sigma = 0.1, lambda = 1,
 * anderson = SPOCK_AA_AUTO. */
void spock_settings_default(spock_settings* s);

typedef struct {
  int32_t status;          /* SPOCK_CONVERGED / SPOCK_MAXITER / SPOCK_NUMERICAL */
  int32_t iters, t_evals;  /* iterations and evaluations of T (= calls of L) */
  int32_t n_k0, n_k1, n_k2, n_km, n_backtracks;
  double xi0, xi;          /* residual xi of section 3 at start and end */
  double V_s0;             /* s^0 of the returned point */
  double V_nested;         /* nested AV@R cost of its (x, u), if requested, else NaN */
  double seconds;          /* host wall time of the call */
  int32_t mapping;         /* lanes per tree family used (8..64), 256 for one workgroup per family,
                              512 for the one-launch dataflow sweeps */
  int32_t flow_fallback;   /* 1 if a bounded wait of the dataflow sweeps gave up (workgroups not
                              all resident): the call was redone from its start with the per-stage
                              form, which the problem keeps from then on; else 0 */
} spock_info;

/* Solves one instance from x0_dev (FP64 [nx], device) and the warm start in
 * v_io_dev. The first solve of a problem times the candidate family-to-lane
 * mappings on its own workspace and keeps the fastest (set the environment
 * variable SPOCK_TEAM to 8, 16, 32, 64 or 256 before factoring to fix it).
 * v_io_dev is [n_v] of the problem precision (zeros for a cold start). On
 * return v_io_dev holds T(v^k) at the last iterate, for which the section-3
 * certificates hold. Synchronises the stream. Errors: SPOCK_EINVAL,
 * SPOCK_EBOX (x0 outside the root box), SPOCK_EHIP, SPOCK_ENOMEM. Not
 * converging is reported in info->status, not as an error. */
int spock_solve(spock_problem* prob, const double* x0_dev, const spock_settings* s,
                void* v_io_dev, spock_info* info_host, void* stream);

/* Solves B independent instances (trees may differ) in one persistent launch
 * captured in a HIP graph: one 256-thread workgroup per instance runs Alg. 3
 * (or CP) to its own termination with no host round trip; the lanes of the
 * workgroup are split into teams, one tree family per team, the team size
 * picked by timing short runs the first time a batch shape is seen (or fixed
 * by the environment variable SPOCK_BATCH_TEAM). probs[b], x0_dev[b] and
 * v_io_dev[b] are as in spock_solve; every problem must have the same
 * precision, nx and nu. infos_host[B] receives the per-instance results
 * (seconds is the wall time of the whole call). The library keeps one device
 * workspace for batched calls (not thread safe). Synchronises the stream.
 * Errors: SPOCK_EINVAL, SPOCK_EHIP, SPOCK_ENOMEM. */
int spock_solve_batched(int32_t B, spock_problem* const* probs,
                        const double* const* x0_dev, const spock_settings* s,
                        void* const* v_io_dev, spock_info* infos_host, void* stream);

/* Gradients of the optimal risk-averse cost V* = s^0 and of the first input
 * u^0 with respect to x0 and the diagonal cost weights, by implicit
 * differentiation at the fixed point v* = T(v*) (section 3): the adjoint
 * w = J_T(v*)' w + g, applied with the transposed CP operator (projection
 * Jacobians at the stored pre-prox point, Alg. 2 sweeps with zero root state
 * for the S1 projection), is solved as (I - J_T(v*)') w = g by restarted
 * GMRES (120 Krylov vectors, 30 when 121 basis vectors would exceed 256 MiB;
 * the environment variable SPOCK_ADJ_RESTART sets
 * 2 to 120), then the parameter Jacobian of T is applied.
 *   v_star_dev: [n_v] of the problem precision, the output of spock_solve
 *   x0_dev: FP64 [nx]; gV: cotangent of V*; gu0_dev: FP64 [nu] cotangent of u^0 or NULL
 *   grad_x0_dev: FP64 [nx] out; grad_q_dev: FP64 [num_nodes][nx] out or NULL
 *     (row c = d/d diag(Q^c), row 0 zero); grad_qN_dev: FP64 [num_nodes][nx]
 *     out or NULL (leaf rows = d/d diag(Q_N^j), other rows zero)
 *   s->eps_abs: tolerance on ||w_{k+1} - w_k||_inf relative to max(1, ||w||_inf);
 *   s->max_iters: cap on applications of J_T'. info->iters, info->xi report
 *   those applications and the last residual |w - J_T' w - g|_inf; info->status is SPOCK_CONVERGED or
 *   SPOCK_MAXITER. Synchronises the stream. The gradient is that of the
 *   fixed point reached; where the solution is not unique (degenerate active
 *   sets) the adjoint may not converge and info->status says so.
 * Errors: SPOCK_EINVAL, SPOCK_EHIP, SPOCK_ENOMEM. */
int spock_backward(spock_problem* prob, const void* v_star_dev, const double* x0_dev, double gV,
                   const double* gu0_dev, double* grad_x0_dev, double* grad_q_dev,
                   double* grad_qN_dev, const spock_settings* s, spock_info* info_host,
                   void* stream);

/* The gradients of spock_backward (section 3, implicit differentiation at
 * the fixed point) for B instances of one problem that differ in x0 and in
 * their solution, at once. The transposed S1 projection of every instance
 * runs as one set of Alg. 2 sweeps over 16-instance matrix-core tiles (the
 * shared-tree form of spock_solve_batched), and the instances' GMRES solves
 * advance in lockstep Arnoldi steps (each its own basis, restart and
 * convergence test, as in spock_backward).
 *   B >= 1; v_star_dev[b], x0_dev[b], grad_x0_dev[b] as in spock_backward
 *   for instance b; gu0_dev: NULL (no u^0 cotangent) or B pointers, each
 *   NULL or FP64 [nu]; grad_q_dev, grad_qN_dev: NULL or B pointers, each
 *   NULL or FP64 [num_nodes][nx]; gV: the same cotangent of V* for all.
 *   info_host[B]: per instance as in spock_backward (info.mapping = 1024).
 * Allocates its workspace (about 121 vectors of n_v per instance, 30 when
 * that would pass 2 GiB) for the call. Synchronises the stream.
 * Errors: SPOCK_EINVAL, SPOCK_EUNSUPPORTED (general risk, polyhedral rows or
 * dense costs), SPOCK_EHIP, SPOCK_ENOMEM; on error no gradient is written. */
int spock_backward_batched(spock_problem* prob, int32_t B, const void* const* v_star_dev,
                           const double* const* x0_dev, double gV, const double* const* gu0_dev,
                           double* const* grad_x0_dev, double* const* grad_q_dev,
                           double* const* grad_qN_dev, const spock_settings* s, spock_info* info_host,
                           void* stream);

/* ---------------------------------------------------------------------------
 * Per-operator entry points (same kernels as the solver; used for operator
 * parity). All vectors are device arrays of the problem precision.
 * ------------------------------------------------------------------------- */
/* eta_dev[n_eta] = L z_dev[n_z] (section 5.2, definition of L) */
int spock_apply_L(spock_problem* prob, const void* z_dev, void* eta_dev, void* stream);
/* z_dev[n_z] = L* eta_dev[n_eta], the adjoint of L */
int spock_apply_Lt(spock_problem* prob, const void* eta_dev, void* z_dev, void* stream);
/* zout_dev = prox_{alpha f}(zin_dev) (section 5.3): s^0 - alpha, projection on
 * S1 with root state x0_dev (Alg. 2), projection on S2. With the dataflow
 * mapping (512) this call and spock_T synchronise the stream to read the
 * sweeps' error word; if a bounded wait gave up they switch the problem to
 * the per-stage form and evaluate again. */
int spock_prox_f(spock_problem* prob, const void* zin_dev, const double* x0_dev,
                 void* zout_dev, void* stream);
/* out_dev = prox_{alpha g*}(w_dev) = w - alpha proj_S3(w / alpha) (section 5.4) */
int spock_prox_gstar(spock_problem* prob, const void* w_dev, void* out_dev, void* stream);
/* Tv_dev = T(v_dev) (eq. chambolle-pock-operator). If stats_host is non-NULL it
 * receives {||xi_p||_inf, ||xi_d||_inf, omega^2, ||r_z||^2, ||r_eta||^2,
 * <r_eta, L r_z>} of r = v - T(v) (section 3, Alg. 3) and the call
 * synchronises. */
int spock_T(spock_problem* prob, const void* v_dev, const double* x0_dev, void* Tv_dev,
            double* stats_host, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): spock_T
 * without any allocation. The sweep buffers and the statistic partials live
 * in a fixed device array of 64 MiB per GPU, held until the process ends;
 * the evaluation always uses the per-stage sweeps (the dataflow form needs
 * buffers of its own). The call allocates nothing: no hipMalloc, hipFree or
 * allocating routine (the caller passes v_dev, x0_dev and Tv_dev). Every
 * call on one GPU shares that GPU's array, so calls that overlap on one GPU
 * (several streams or threads) race; calls ordered on one stream do not.
 * Nothing in the array needs to start cleared. stats_host as in spock_T (the
 * call then synchronises). Errors: SPOCK_EINVAL, SPOCK_ETOOBIG (the problem's
 * buffers exceed the 64 MiB), SPOCK_EUNSUPPORTED (device index 64 or above),
 * SPOCK_EHIP. */
int spock_T_noalloc(spock_problem* prob, const void* v_dev, const double* x0_dev, void* Tv_dev,
                    double* stats_host, void* stream);

/* Timing aid for the CP operator (results as spock_T, statistics not
 * returned): evaluates T(v_dev) reps times on `stream` with HIP events
 * recorded between its phases and writes the mean duration in microseconds
 * of each phase to us_out_host[0..4]: pre-pass (xbar, ubar, S2), both Alg. 2
 * sweeps, post-pass (dual update and statistics), reduction of the
 * statistics, whole evaluation. Synchronises. reps must be >= 1. */
int spock_profile_T(spock_problem* prob, const void* v_dev, const double* x0_dev, void* Tv_dev,
                    int32_t reps, double* us_out_host, void* stream);

/* Library version string */
const char* spock_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPOCK_H */
