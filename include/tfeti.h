/*
 * tfeti.h - C ABI of the MI355X (gfx950) TFETI semismooth-Newton solver for
 * elastoplasticity with von Mises yield and linear isotropic hardening.
 *
 * Method: Cermak, Kozubek, Sysala, Valdman, "A TFETI Domain Decomposition
 * Solver for Elastoplastic Problems".  Implicit Euler in time (Section 2.4),
 * Q1-hexahedron FEM in space, semismooth Newton per load step (Algorithms 2
 * and 4), each linearized system solved by Total FETI with the projected
 * preconditioned conjugate gradient method PCGP (Algorithm 3).
 *
 * Conventions shared by every call:
 *  - Every function returns an int status: TFETI_OK (0), TFETI_CONVERGED (1,
 *    Newton only), a warning (>= 2, results valid) or an error (< 0, outputs
 *    undefined).  No C++ exception crosses the ABI; tfeti_last_error() gives
 *    a message for the last failing call on a handle.
 *  - Array arguments are DEVICE pointers unless the name ends in _host.  The
 *    caller owns every buffer it passes; none is retained after return.  The
 *    handle owns all of its internal device memory.
 *  - Work is enqueued on the HIP stream given to tfeti_setup (a hipStream_t
 *    passed as void*; NULL is the null stream).  Calls are ordered on that
 *    stream; report structs are filled synchronously (the call waits for its
 *    own work before filling them).
 *  - A handle is not thread safe: calls on one handle must not overlap.
 *
 * Numbering (bit-exact with the test oracle):
 *  - global node (i,j,k) -> i + (Nx+1)*(j + (Ny+1)*k); subdomains are the
 *    boxes (I,J,K) that are not absent, numbered in the order of
 *    I + Sx*(J + Sy*K) (so p = I + Sx*(J + Sy*K) when none is absent); local
 *    nodes and elements lexicographic, x fastest.  Untorn (global) DOF
 *    vectors cover the nodes that belong to some subdomain, node ascending.
 *  - torn vectors (length n_torn) stack the subdomain vectors in subdomain
 *    order; the local DOF of (local node a, component c) is 3a + c.
 *  - Gauss-point state arrays are ordered subdomain, local element, Gauss
 *    point (2x2x2 rule, xi fastest); stresses are Voigt vectors
 *    (s11, s22, s33, s12, s23, s13), strains use engineering shears
 *    (e11, e22, e33, 2e12, 2e23, 2e13) (Section 3.1, vector form).
 *  - multipliers (length m) are ordered as the rows of B = [B_G; B_U]
 *    (Section 4.1), orthonormal form: for each (global node, component) with
 *    copies in subdomains p1 < ... < pk, a Dirichlet-constrained pair gives k
 *    rows of B_U (one +1 per copy) and no B_G row; otherwise k-1 Helmert rows
 *    j = 1..k-1 with +c_j at p1..pj and -j*c_j at p(j+1), c_j = 1/sqrt(j(j+1)).
 *    B_G rows come first (node ascending, component, j), then B_U rows (node
 *    ascending, component, copy ascending).
 */
#ifndef TFETI_H
#define TFETI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TFETI_OK 0
#define TFETI_CONVERGED 1            /* Newton: the load step has converged    */
#define TFETI_W_PCG_MAXIT 2          /* PCGP stopped at max_pcg iterations     */
#define TFETI_W_NEWTON_MAXIT 3       /* Newton reached max_newton iterations   */
#define TFETI_W_WARMSTART_REJECTED 4 /* a warm start was non-finite; cold used */
#define TFETI_E_INVALID (-1)         /* bad argument, size or call order       */
#define TFETI_E_HIP (-2)             /* a HIP runtime call failed              */
#define TFETI_E_OOM (-3)             /* device allocation failed               */
#define TFETI_E_NOT_SPD (-4)         /* a Cholesky pivot was <= 0 or not finite*/

/* ---- problem description (host struct) -------------------------------- */
typedef struct {
  double E, nu;        /* Young modulus, Poisson ratio (Hooke law, Section 2.2) */
  double sigma_y, H;   /* initial yield stress and hardening modulus H_m > 0    */
} tfeti_material;

typedef struct {
  int32_t S[3];                 /* subdomains per axis (box decomposition)      */
  const int32_t* n_host[3];     /* n_host[a][I]: elements of slab I along axis a */
  double extent[3];             /* box edge lengths; elements are uniform per axis*/
  tfeti_material mat;
  int32_t dirichlet[6][3];      /* [face][comp] != 0: u_comp = 0 on that face;
                                   faces x=0, x=X, y=0, y=Y, z=0, z=Z           */
  double traction[6][3];        /* traction vector on each face at load factor 1 */
  const uint8_t* absent_host;   /* NULL, or S[0]*S[1]*S[2] flags at I + S[0]*(J +
                                   S[1]*K): nonzero leaves box (I,J,K) out of the
                                   body (a hole or notch through the box
                                   decomposition); faces it exposes are free    */
} tfeti_problem;

/* ---- solver options (host struct) ------------------------------------- */
#define TFETI_PREC_FP64 0       /* FP64 factors and F-applies                   */
#define TFETI_PREC_FP32 1       /* FP32 factors and F-applies, FP64 outer dual
                                   refinement; FP64 coarse solve, inner products
                                   and return map                               */
typedef struct {
  int32_t precision;            /* TFETI_PREC_*                                 */
  int32_t preconditioner;       /* 0 none, 1 lumped B K B^T, 2 Dirichlet
                                   Bbar Sbar Bbar^T (Section 4.2): Sbar the Schur
                                   complement of the unregularized tangent onto
                                   the DOFs of the nodes carrying rows of B,
                                   applied through banded Cholesky factors of
                                   the interior blocks K_ii (the interior nodes
                                   of a box subdomain form a box; factors in
                                   FP64, solved in the F-apply's precision)     */
  double eps_pcg;               /* PCGP relative tolerance                      */
  double eps_newton;            /* Newton relative-residual tolerance           */
  int32_t max_pcg;              /* PCGP iteration cap (default 5000)            */
  int32_t max_newton;           /* Newton iteration cap per load step (50)      */
  int32_t warm_start;           /* 0 cold; 1 warm.  First Newton iteration of a
                                   load step: the previous step's first-iteration
                                   lambda scaled by the load-increment ratio.
                                   Later iterations: the previous iteration's
                                   lambda and, while it keeps winning, the
                                   learned candidate if one is set; the
                                   one with the smaller projected initial residual
                                   is used, and cold start if both are not finite */
  int32_t use_graph;            /* replay the PCGP iteration as a HIP graph     */
  int32_t tile;                 /* factor tile rows 16/32/64; 0 = autotuned: at
                                   the first factorization, every tile 16/32/64
                                   with either subdomain order and 256, 512 or
                                   1024 threads per subdomain is timed (median
                                   of 20 F-applies x 70 + one panel packing) and
                                   the cheapest is kept;
                                   the choice is cached in the file named by the
                                   environment variable TFETI_AUTOTUNE_CACHE (if
                                   set), keyed by GPU architecture, precision and
                                   subdomain-size histogram                      */
  double refine_eps;            /* FP32 mode: smallest inner PCGP tolerance
                                   relative to the outer residual (0 = 1e-5);
                                   each sweep aims at half the reduction still
                                   needed, but not below this                    */
  int32_t check_every;          /* host polls convergence every N iterations    */
  int32_t refactor_all;         /* 1: factorize every subdomain each Newton
                                   iteration; 0: keep the factor of a subdomain
                                   whose tangent is and was the elastic one      */
  int32_t fapply_format;        /* F-applies inside the PCGP loop (and
                                   tfeti_fapply) through TFETI_FAPPLY_FACTORS,
                                   TFETI_FAPPLY_EXPLICIT or TFETI_FAPPLY_HYBRID */
  int32_t pad;
} tfeti_options;
#define TFETI_FAPPLY_FACTORS 0  /* forward and backward substitution with the
                                   packed Cholesky factors (Remark 1 in Section
                                   4.2)                                         */
#define TFETI_FAPPLY_EXPLICIT 1 /* explicit local dual operators: per subdomain
                                   the block of K_reg^{-1} on the DOFs that
                                   carry rows of B, formed on the matrix cores
                                   from the FP64 factor whenever the subdomain
                                   is factorized (or its elastic factor is
                                   copied back), stored as the lower triangle in
                                   the F-apply's precision and applied as one
                                   symmetric product; d, lambda_Im, the FP32
                                   outer refinement and u keep the factors      */
#define TFETI_FAPPLY_HYBRID 2   /* in one launch, the explicit local dual
                                   operators of the subdomains that keep the
                                   factor of their elastic tangent (formed when
                                   that factor is, copied back with it) and
                                   the factor sweeps of the others; without
                                   kept factors (refactor_all) the factor path */

/* ---- reports (host structs) ------------------------------------------- */
typedef struct {
  int32_t iters;                /* PCGP iterations (F-applies inside the loop)  */
  int32_t fapplies;             /* all F-applies of the solve                   */
  int32_t converged;            /* 1 if ||P r|| <= eps * r_ref                  */
  int32_t outer;                /* FP32 mode: outer refinement sweeps           */
  double r_ref;                 /* ||P (d - F lambda_Im)||                      */
  double r_final;               /* last ||P r||                                 */
  double ms;                    /* wall time of the call                        */
  int32_t warm_choice;          /* 0 cold start, 1 first guess, 2 second guess   */
  int32_t pad;
} tfeti_pcg_report;

typedef struct {
  int32_t iteration;            /* Newton iteration index i (1-based)           */
  int32_t pcg_iters;
  int32_t fapplies;
  int32_t plastic_gp;           /* Gauss points on the plastic branch           */
  int32_t plastic_elements;     /* elements with at least one plastic point     */
  double relres;                /* ||assembled residual|| / ||assembled df||, free DOFs */
  double crit;                  /* the paper's increment criterion (Algorithm 2)*/
  double ms_assembly, ms_factor, ms_pcg, ms_total;
  int32_t warm_choice;          /* 0 cold, 1 fallback lambda, 2 learned         */
  int32_t refactored;           /* subdomains factorized in this iteration (the
                                   others kept the factor of their unchanged
                                   elastic tangent)                              */
  int32_t restored;             /* subdomains elastic again whose elastic factor
                                   was copied back instead of factorized (the
                                   library keeps every subdomain's elastic
                                   factor once all were elastic at one
                                   factorization; not with refactor_all)         */
  int32_t pad;
} tfeti_newton_report;

typedef struct {
  int64_t n_sub, n_torn, m, m_G, m_U, l, n_elem, n_gp, n_gdof;
  int64_t skyline_entries;      /* sum over subdomains of the factor envelope    */
  int64_t factor_entries;       /* stored entries of one factor layout           */
  int64_t factor_bytes;         /* bytes read by one pass over all factors       */
  int32_t tile;                 /* factor tile rows in use                       */
  int32_t precision;
  int32_t schedule;             /* subdomain order of the solve launch: 0 longest
                                   first, 1 natural                              */
  int32_t autotuned;            /* 0 tile fixed by the options, 1 searched by the
                                   autotuner, 2 taken from its cache             */
  int32_t threads;              /* threads per workgroup of the subdomain solves
                                   (256; 512 or 1024 when the autotuner finds
                                   them faster: few or uneven subdomains per
                                   compute unit)                                 */
  int32_t pad;
  int64_t explicit_bytes;       /* bytes one explicit F-apply reads of the local
                                   operators (0 unless TFETI_FAPPLY_EXPLICIT)    */
} tfeti_sizes;

typedef struct tfeti_handle tfeti_handle;

/* ---- lifetime ---------------------------------------------------------- */

/* Build the decomposition, the gluing matrix B (Section 4.1), the rigid body
 * modes R (orthonormal kernel basis, Section 4.2), G = R^T B^T, the coarse
 * matrix G G^T and its inverse (factorized once on the device: R and B are
 * fixed for the whole run), and allocate every device buffer.  State starts
 * at zero (Algorithm 4, initial step).  Errors: TFETI_E_INVALID for
 * non-positive sizes, null pointers or E, H, sigma_y <= 0; TFETI_E_OOM. */
int tfeti_setup(const tfeti_problem* prob_host, const tfeti_options* opt_host,
                void* stream, tfeti_handle** out);
void tfeti_destroy(tfeti_handle* h);
/* h NULL: the message of the last failed handle-less call on this thread. */
const char* tfeti_last_error(const tfeti_handle* h);
int tfeti_get_sizes(const tfeti_handle* h, tfeti_sizes* out_host);

/* Copy B in CSR form to host buffers of m+1, nnz, nnz entries: row pointers,
 * torn DOF of each entry, coefficient.  Any pointer may be NULL (then only
 * *nnz_host is written).  Used to check the index maps bit for bit. */
int tfeti_get_B_host(const tfeti_handle* h, int64_t* nnz_host, int64_t* rowptr_host,
                     int64_t* col_host, double* val_host);

/* ---- time stepping (Algorithms 1 and 4) -------------------------------- */

/* Start load step k -> k+1: the load increment is dload_factor times the
 * load at factor 1, and the displacement increment restarts at zero. */
int tfeti_begin_load_step(tfeti_handle* h, double dload_factor);

/* One Newton iteration i of the current load step (Algorithm 4 body):
 * return map at every Gauss point, internal force and tangent assembly
 * (Algorithm 5), residual f = df - f_int.  For i >= 2, if the relative
 * residual of the assembled system on free DOFs is <= eps_newton, returns
 * TFETI_CONVERGED without solving.  Otherwise regularizes and factorizes the
 * subdomain tangents, solves the dual problem by PCGP (Algorithm 3) and
 * updates the displacement increment.  Returns TFETI_W_NEWTON_MAXIT after
 * max_newton iterations, TFETI_E_NOT_SPD on a failed factorization. */
int tfeti_newton_step(tfeti_handle* h, tfeti_newton_report* rep_host);

/* Commit the load step: u += du, sigma += dsigma, kappa += dkappa, with the
 * increments evaluated at the converged displacement increment
 * (Algorithm 4, end of the time step). */
int tfeti_commit_load_step(tfeti_handle* h);

/* ---- dual solver (Algorithm 3) ----------------------------------------- */

/* Solve min 1/2 v^T K v - f^T v subject to B v = 0 (Section 4.1) for the
 * currently factorized K by PCGP: lambda_Im = G^T (G G^T)^{-1} R^T f,
 * d = B K^+ f, projected iterations on Ker G, alpha = -(G G^T)^{-1} G r,
 * u = K^+ (f - B^T lambda) + R alpha.  f and u_out: n_torn FP64; lambda_guess
 * (m, may be NULL) warm start, used as lambda_Im + P lambda_guess;
 * lambda_out: m FP64.  Stop: ||P r|| <= eps_pcg ||P(d - F lambda_Im)||.
 * Returns TFETI_W_PCG_MAXIT if the cap was reached. */
int tfeti_dual_pcg(tfeti_handle* h, const double* f, const double* lambda_guess,
                   double* lambda_out, double* u_out, tfeti_pcg_report* rep_host);

/* ---- building blocks (used by tests and benchmarks) -------------------- */

/* Return map, internal force and tangent assembly at displacement increment
 * du (n_torn, FP64, device) against the committed state; writes the torn
 * internal force sum_T sum_g w_g B_g^T dsigma_g to fint (n_torn) and keeps
 * the tangent inside the handle.  If plastic_count_host != NULL it receives
 * the number of plastic Gauss points. */
int tfeti_assemble(tfeti_handle* h, const double* du, double* fint, int64_t* plastic_count_host);

/* Regularize (fixing nodes, Remark 1) and factorize the assembled tangents
 * (of the subdomains that have a plastic Gauss point or whose factor is not
 * of the elastic tangent, unless options.refactor_all).  TFETI_E_NOT_SPD if
 * a pivot is <= 0 or not finite; the factorized bands are then unusable and
 * every further call fails the same way until tfeti_assemble (or a Newton
 * step) forms a new tangent. */
int tfeti_factorize(tfeti_handle* h);

/* q = F lambda = B K^+ B^T lambda (m -> m, FP64) with the current factors in
 * the factor precision; the fused per-subdomain solve plus the B gather. */
int tfeti_fapply(tfeti_handle* h, const double* lambda, double* q);

/* y = K_reg^{-1} x on a torn vector (n_torn, FP64) with the current factors. */
int tfeti_kplus(tfeti_handle* h, const double* x, double* y);

/* out = P w = w - G^T (G G^T)^{-1} G w (m -> m, FP64). */
int tfeti_project(tfeti_handle* h, const double* w, double* out);

/* out = the handle's preconditioner applied to w (m -> m, FP64): B K B^T w
 * with the unregularized tangent (lumped), or Bbar Sbar Bbar^T w
 * (Dirichlet, options.preconditioner = 2; needs a factorization).  With
 * preconditioner 0 the lumped product. */
int tfeti_precondition(tfeti_handle* h, const double* w, double* out);

/* State access: sigma (n_gp*6), kappa (n_gp), u (n_torn), du (n_torn),
 * dsigma (n_gp*6), dkappa (n_gp), plastic (n_gp, uint8); NULL skips. */
int tfeti_get_state(const tfeti_handle* h, double* sigma, double* kappa, double* u,
                    double* du, double* dsigma, double* dkappa, uint8_t* plastic);
int tfeti_set_state(tfeti_handle* h, const double* sigma, const double* kappa,
                    const double* u, const double* du);

/* Multipliers of the last PCGP solve (m, FP64, device). */
int tfeti_get_lambda(const tfeti_handle* h, double* lambda);

/* Timing of the dominant kernel: when on, F-apply subdomain-solve kernels
 * are bracketed by HIP events on the stream they run on (inside a replayed
 * PCGP graph, those of one graph batch in four, the rest replay a graph
 * without event nodes); get returns the summed milliseconds and the number
 * of timed kernels that did work since the last set (set also resets the
 * totals). */
int tfeti_set_timing(tfeti_handle* h, int on);
int tfeti_get_timing(tfeti_handle* h, double* ms_host, int64_t* count_host);
/* Algorithmic bytes of the F-apply kernels counted by tfeti_get_timing since
 * timing was switched on: per launch, both triangular sweeps over the
 * envelope of each factor the launch solves with, plus the stored tiles of
 * each explicit operator it applies (with TFETI_FAPPLY_HYBRID the mix of
 * the factorization in use).  Section 4.2 (F = B K^+ B^T). */
int tfeti_get_timing_bytes(tfeti_handle* h, double* bytes_host);

/* Graph replay state of the PCGP iteration: 0 not captured (yet or option
 * off), 1 replaying a captured graph, 2 capture failed (eager launches). */
int tfeti_graph_status(const tfeti_handle* h);

/* Host-only (no device work): build the model of prob and report its sizes
 * (factor_bytes and precision are not set) and, when the pointers are not
 * NULL, B in CSR like tfeti_get_B_host (host buffers of m+1, nnz, nnz).  Lets
 * the index maps be checked without a GPU.  tile: 0, 16, 32 or 64.  Errors:
 * TFETI_E_INVALID, the reason in tfeti_last_error(NULL). */
int tfeti_model_host(const tfeti_problem* prob_host, int32_t tile, tfeti_sizes* sizes_host, int64_t* nnz_host,
                     int64_t* rowptr_host, int64_t* col_host, double* val_host);

/* ---- learned warm start: network kernels ------------------------------- */

/* A 3-layer perceptron h1 = relu(x W1^T + b1), h2 = relu(h1 W2^T + b2),
 * y = h2 W3^T + b3 with FP32 master weights, bfloat16 copies used by the
 * products and bfloat16 activations, FP32 accumulation.  All pointers are
 * device buffers owned by the caller; W[l] is row-major (out x in). */
typedef struct {
  int32_t d_in, d_h, d_out;     /* 31, 256, 21 for the warm start            */
  float* W[3];                  /* master weights                            */
  float* b[3];
  uint16_t* Wb[3];              /* bfloat16 copies of W                      */
  float* gW[3];                 /* gradients (written by tfeti_mlp_loss_grad) */
  float* gb[3];
  float* mW[3];                 /* Adam first and second moments             */
  float* vW[3];
  float* mb[3];
  float* vb[3];
} tfeti_mlp;

/* Floats of device workspace needed for a batch of n rows. */
int tfeti_mlp_work_size(const tfeti_mlp* net_host, int64_t n, int64_t* floats_host);
/* Wb = bf16(W) (after initializing or loading W). */
int tfeti_mlp_sync_bf16(const tfeti_mlp* net_host, void* stream);
/* Y (n x d_out, FP32) = network(X (n x d_in, FP32, rounded to bf16)). */
int tfeti_mlp_forward(const tfeti_mlp* net_host, int64_t n, const float* X, float* Y, float* work, void* stream);
/* The forward pass of tfeti_mlp_forward without a workspace argument and
 * without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Its scratch (the bf16 inputs and both hidden layers) is a
 * fixed device array of 8 MiB per GPU, held until the process ends: n rows
 * need 4 ((n d_in + 1)/2 + 2 ((n d_h + 1)/2)) bytes, so about 7700 rows of
 * the 31 -> 256 -> 256 -> 21 warm-start network per call; larger n is
 * rejected with TFETI_E_INVALID (message in tfeti_last_error(NULL)) and
 * must be split.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (other streams, other threads) race.  Nothing in it
 * needs to start at zero.  Results are bitwise those of tfeti_mlp_forward. */
int tfeti_mlp_forward_noalloc(const tfeti_mlp* net_host, int64_t n, const float* X, float* Y, void* stream);
/* Forward, masked mean squared error L = 1/(2n) sum M (Y - T)^2 into *loss
 * (device scalar), and the gradients of L into gW, gb. */
int tfeti_mlp_loss_grad(const tfeti_mlp* net_host, int64_t n, const float* X, const float* T, const float* M,
                        float* Y, float* loss, float* work, void* stream);
/* One Adam step (step = 1, 2, ...) on W, b from gW, gb; refreshes Wb. */
int tfeti_mlp_adam(const tfeti_mlp* net_host, int32_t step, float lr, float beta1, float beta2, float eps,
                   void* stream);

/* ---- learned warm start: features, targets and candidate ------------- */

/* The interface nodes (mesh nodes carrying multiplier rows) of the handle's
 * model; each holds up to 21 rows: 7 slots per displacement component (the
 * orthonormal gluing rows of a node shared by up to 8 subdomains, or one
 * Dirichlet row per copy).  s_lam = |dload| * |traction at factor 1| * element
 * face area of the loaded face is the nodal force scale of a load increment
 * dload (1 if zero).  Buffers below are device memory owned by the caller and
 * work on the handle's stream; they are asynchronous. */
int tfeti_warm_nodes(const tfeti_handle* h, int64_t* n_host);
/* X (n x 31, FP32): load direction (3), lambda_prev of the node's rows / s_lam
 * (21, 0 on empty slots), mean committed hardening kappa of the elements around
 * the node times H/sigma_y (1), one-hot node class (6: gluing over 2/4/8
 * copies, Dirichlet with 1/2/4 copies).  lambda_prev (m) may be NULL (zero).
 * M (n x 21, may be NULL) receives 1 on used slots, 0 on empty ones. */
int tfeti_warm_features(tfeti_handle* h, const double* lambda_prev, double dload, float* X, float* M);
/* T (n x 21, FP32) = (lambda_next - lambda_prev) / s_lam on used slots, 0 else. */
int tfeti_warm_targets(tfeti_handle* h, const double* lambda_prev, const double* lambda_next, double dload,
                       float* T);
/* lambda_out (m) = lambda_prev + s_lam * Y on every row (Y: n x 21 FP32). */
int tfeti_warm_candidate(tfeti_handle* h, const double* lambda_prev, const float* Y, double dload,
                         double* lambda_out);
/* Offer lambda (m, device, copied) as the second warm-start candidate at the
 * Newton iterations i >= 2 of the current (or next) load step, until it loses
 * to the previous iteration's multipliers once; NULL withdraws it.
 * tfeti_commit_load_step clears it; used only when warm_start is on. */
int tfeti_set_learned_guess(tfeti_handle* h, const double* lambda);
/* Multipliers of the final Newton iteration of the last committed load step
 * (m, device): the interface-force increment of that step.  *available_host = 0
 * and zeros if none was committed yet. */
int tfeti_get_converged_lambda(const tfeti_handle* h, double* lambda, int32_t* available_host);

/* ---- stateless return map (Section 2.4, Voigt form of Section 3.1) ----- */

/* For npts points: trial = sigma_k + C deps; if Phi(trial, kappa_k) <=
 * 1e-12 (sigma_y + H kappa_k) (a committed point on the yield surface counts
 * as elastic whatever the sign of its rounding) the step is elastic (dsigma = C deps, dkappa = 0, D = C); otherwise
 * dkappa = Phi/(3mu+H), dsigma = C deps - 3mu/(3mu+H) sqrt(2/3) Phi n with n
 * the unit deviator of the trial stress, and D the generalized derivative
 * C - 2mu beta E_eps - 2mu beta sqrt(2/3) (sigma_y + H kappa_k)/|dev trial|
 * (n n^T - E_eps), beta = 3mu/(3mu+H).  sigma_k, deps, dsigma: 6*npts;
 * kappa_k, dkappa: npts; Dtan: 36*npts row-major or NULL; plastic: npts
 * bytes or NULL.  All device pointers, FP64.  Errors: TFETI_E_INVALID. */
int return_map(const tfeti_material* mat_host, int64_t npts, const double* sigma_k,
               const double* kappa_k, const double* deps, double* dsigma, double* dkappa,
               double* Dtan, uint8_t* plastic, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TFETI_H */
