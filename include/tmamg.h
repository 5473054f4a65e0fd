/*
 * tmamg — DD-alpha-AMG solver for the twisted-mass clover Wilson operator
 * on AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The operator (arXiv:1710.06198, Sec. 1 and Sec. 1.1) is
 *     D(mu) = D + i mu Gamma5,
 * with D the clover-improved Wilson operator in m0-normalisation:
 *     D(mu) psi(x) = A(x) psi(x) + i mu g5 psi(x)
 *        - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)],
 *     A(x) = (m0 + 4) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *     m0 = 1/(2 kappa) - 4,
 * chiral gamma basis (g5 = diag(1,1,-1,-1)), periodic space, antiperiodic
 * time (optional).  The solver is the multigrid-preconditioned flexible
 * Krylov method of Sec. 1.1, Eq. (1): post-smoothing by k sweeps of SAP,
 * aggregation-based P from N_v adaptively built test vectors (Gamma5-
 * compatible: Gamma5 P = P Gamma5,c), Galerkin D_c = P^dag D P and the
 * coarse twisted-mass operator D_c(+-mu) = D_c +- i mu Gamma5,c with one P
 * for both signs of mu.
 *
 * Buffers.  Every field pointer is DEVICE memory owned by the caller and
 * valid for the duration of the call; the library copies what it keeps.
 * Canonical layouts (complex128 = two doubles, x fastest):
 *   gauge links   [4][T][Z][Y][X][3][3]      mu = 0..3 <-> x, y, z, t
 *   spinor fields [n][T][Z][Y][X][4][3]      spin-colour index spin*3 + colour
 *   force         [4][T][Z][Y][X][3][3]      traceless anti-Hermitian
 *   coarse fields [n][Tc][Zc][Yc][Xc][d]     d = 2 N_v, index s*N_v + i
 * Host pointers are marked "host".
 *
 * Ordering.  All work is ordered on the stream given at creation; every
 * call returns after synchronising that stream (status and info are host
 * values).  Inputs are read on that stream: device data written on another
 * stream must be complete, or ordered before the call (an event that the
 * context's stream waits on); the Python binding orders the context's
 * stream after the caller's current stream on every call.  A context is not
 * thread-safe.
 *
 * Errors.  Negative status: outputs undefined, tmamg_last_error() holds a
 * message.  TMAMG_NOT_CONVERGED: x holds the best iterate and
 * info.true_rel_resid its FP64 true residual.
 */
#ifndef TMAMG_H
#define TMAMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmamg_ctx tmamg_ctx;

typedef enum {
  TMAMG_OK = 0,
  TMAMG_NOT_CONVERGED = 1,
  TMAMG_EINVAL = -1,     /* bad argument or parameter combination */
  TMAMG_ENOMEM = -2,     /* device allocation failed */
  TMAMG_EHIP = -3,       /* HIP runtime error */
  TMAMG_ENUMERIC = -4,   /* NaN/Inf in input or breakdown */
  TMAMG_ESTATE = -5      /* call order: e.g. solve before setup */
} tmamg_status;

enum { TMAMG_FP64 = 0, TMAMG_MIXED = 1 };                                          /* precision */
enum { TMAMG_STORE_FP64 = 0, TMAMG_STORE_FP32 = 1, TMAMG_STORE_BF16 = 2, TMAMG_STORE_FP16 = 3 }; /* P, D_c */

typedef struct {
  int dims[4];          /* Lx, Ly, Lz, Lt */
  int t_antiperiodic;   /* 1: fermion field antiperiodic in time */
} tmamg_lattice;

typedef struct {
  int nlevels;          /* 1 (SAP only), 2 or 3 */
  int agg[2][4];        /* aggregate shape per coarsening; agg[0] is also the fine SAP block */
  int nv[2];            /* test vectors per coarsening (<= 64) */
  int setup_iters;      /* adaptive setup iterations (v_i <- B v_i) */
  int init_smooth;      /* smoother applications in the initial setup phase */
  int sap_block1[4];    /* SAP block on the first coarse level (3 levels) */
  int sap_sweeps[2];    /* k: SAP sweeps on the fine / first coarse level */
  int mr_steps;         /* minimal-residual steps per SAP block solve */
  int l2_iters;         /* FGMRES steps on the intermediate level (3 levels) */
  double l2_tol;        /* its relative tolerance */
  int coarsest_iters;   /* GMRES steps on the coarsest level */
  double coarsest_tol;  /* its relative tolerance */
  int restart;          /* outer FGMRES restart length (<= 127) */
  int max_iter;         /* outer iteration limit (all cycles) */
  int precision;        /* TMAMG_FP64 or TMAMG_MIXED */
  int storage;          /* TMAMG_STORE_*: P and D_c storage in mixed precision */
  double inner_tol;     /* mixed: relative reduction per FP32 inner cycle */
  unsigned long long seed;  /* test-vector noise */
  int use_graph;        /* 1: with three levels, the intermediate-level solve of
                           every fine cycle is captured once per right-hand-side
                           count as a HIP graph and replayed (same kernels, same
                           order, identical results); 0: plain launches */
  int nd_coarse_coupling;  /* doublet solves (Sec. 1.1, Eq. (2)): 1 (default) the coarse
                              levels solve D_ND,c = P_ND^dag D_ND P_ND, i.e. each flavour's
                              D_c(+-mubar) coupled by -epsbar; 0: each flavour's own cycle */
  int setup_chunk;      /* memory plan: test vectors the setup smooths and cycles at once on
                           each level (0: all of them); the setup's fine work buffer holds
                           this many vectors.  The result does not depend on it: every test
                           vector is treated alone */
  int keep_test_vectors;  /* memory plan: 1 (default) keep the fine test vectors after the setup
                             for tmamg_setup_update; 0 release them (and the setup's work
                             buffers), tmamg_setup_update then returns TMAMG_ESTATE */
} tmamg_params;

typedef struct {
  int status;              /* tmamg_status of the call */
  int outer_iters;         /* FGMRES iterations summed over cycles */
  int cycles;              /* restart cycles / reliable updates */
  double true_rel_resid;   /* max over right-hand sides of ||b - D x|| / ||b|| (FP64);
                              tmamg_solve_shifted: of ||b - (D D^dag + sigma) x|| / ||b|| */
  double t_setup_s;        /* last setup */
  double t_solve_s;        /* this call */
  long long l2_iters_total;       /* intermediate-level FGMRES steps in this call, summed over
                                     its calls (a batch's step counts once) */
  long long coarsest_iters_total; /* coarsest-level GMRES iterations in this call, summed over
                                     calls and right-hand sides */
} tmamg_info;

/* Device memory for a context's internal buffers (optional, see
 * tmamg_create).  alloc returns `bytes` of device memory usable on
 * hip_stream, or NULL when it cannot (the call then fails with
 * TMAMG_ENOMEM); free releases a pointer alloc returned.  `user` is passed
 * through.  Both are called only from inside the library's own calls on
 * that context, on the calling thread. */
typedef void* (*tmamg_alloc_fn)(size_t bytes, void* hip_stream, void* user);
typedef void (*tmamg_free_fn)(void* ptr, void* hip_stream, void* user);
typedef struct {
  tmamg_alloc_fn alloc;
  tmamg_free_fn free;
  void* user;
} tmamg_allocator;

/* Fill *p with the defaults (2 levels, 4^4 aggregates, N_v = 12, 3 setup
 * iterations, SAP k = 4 with 4 MR steps, FGMRES(30), FP64): the method's
 * parameters of Sec. 1.1, which the paper does not print (plumbing). */
tmamg_status tmamg_default_params(tmamg_params* p);

/* Create a context for one lattice (the lattice and multigrid parameters
 * of Sec. 1.1; the paper's runs use three levels, Sec. 1.2).  hip_stream: a
 * hipStream_t (NULL = the null stream).  allocator: host, may be NULL
 * (hipMalloc/hipFree); when given, every internal device buffer of the
 * context comes from allocator->alloc and goes back through
 * allocator->free, at the latest in tmamg_destroy; the struct is copied.
 * Lattice extents must be multiples of agg[0] (and agg[1] on the coarse
 * lattice); SAP needs an even number of blocks (or one) per dimension on
 * every smoothed level.  *ctx is NULL on error. */
tmamg_status tmamg_create(tmamg_ctx** ctx, const tmamg_lattice* lat, const tmamg_params* par, void* hip_stream,
                          const tmamg_allocator* allocator);

/* Setup (Sec. 1.1 adaptive setup): copy the links U (device, canonical
 * complex128), build the clover term for c_sw and m0 = 1/(2 kappa) - 4,
 * then build the hierarchy at twisted mass mu: random test vectors,
 * init_smooth smoother applications, setup_iters iterations of
 * v_i <- B_MG v_i, Gram-Schmidt per aggregate and chirality (FP64), P and
 * D_c.  Links must be SU(3) within 1e-6 (TMAMG_ENUMERIC otherwise). */
tmamg_status tmamg_setup(tmamg_ctx* ctx, const void* U, double kappa, double csw, double mu);

/* Setup update on new links U (same kappa, c_sw, mu), Sec. 2 (setup
 * updates along the molecular-dynamics trajectory, one setup iteration per
 * update): P and D_c are rebuilt on U from the kept test vectors, which
 * then take `iters` further setup iterations.  U: device, canonical; the
 * same SU(3) check and errors as tmamg_setup; TMAMG_ESTATE before a
 * setup or when the setup released its test vectors (keep_test_vectors
 * = 0). */
tmamg_status tmamg_setup_update(tmamg_ctx* ctx, const void* U, int iters);

/* Solve D(mu_r) x_r = b_r for r < nrhs, in one batch: FGMRES
 * right-preconditioned by the multigrid cycle of Sec. 1.1, Eq. (1), with
 * D(-mu) through the same P (Sec. 1.1, D_c(+-mu) = D_c +- i mu Gamma5,c).
 * b, x: device, canonical spinors [nrhs] (may not alias).  mu_rhs: host
 * [nrhs] signed twisted masses, or NULL for the setup mu on every
 * right-hand side.  Stops when every ||b_r - D x_r|| / ||b_r|| <= tol (FP64
 * true residual), 0 < tol < 1.  A zero b_r gives x_r = 0.  TMAMG_ESTATE
 * before a setup; TMAMG_ENUMERIC for NaN/Inf in b; TMAMG_EHIP also when a
 * persistent coarse kernel's bounded barrier wait gave up (x still holds
 * the iterate the FP64 residual in info describes; the context then stops
 * using those kernels). */
tmamg_status tmamg_solve(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                         tmamg_info* info);

/* tmamg_solve from an initial guess: on entry x holds x0_r (device,
 * canonical [nrhs]); the first FP64 residual is b - D x0.  A right-hand side
 * whose initial residual exceeds ||b_r|| starts from zero instead.  Used for
 * the first-order initial guesses of shifted systems (Sec. 3, Eq. (6): an
 * expansion of the shifted inverse in the shift). */
tmamg_status tmamg_solve_guess(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                               tmamg_info* info);

/* Squared / shifted systems (D D^dag + sigma_r) x_r = b_r with one
 * hierarchy (the two-step solves of Sec. 1.1 for D^dag D, and the shifted
 * systems of the Hasenbusch monomials, Eq. (3), and of the rational
 * approximation, Eq. (5)): since D D^dag + sigma = D(mu') D(mu')^dag with
 * mu' = sqrt(mu^2 + sigma), solve D(mu') w = b, then
 * x = Gamma5 D(-mu')^-1 Gamma5 w, each step to tol; the FP64 residual of
 * the shifted system itself is then checked and, while above tol, the pair
 * of solves is repeated on it (defect correction, at most three passes).
 * sigma: host [nrhs] (>= 0; sigma = 0 gives D D^dag).  b, x: device
 * canonical [nrhs]; info.true_rel_resid is the shifted system's residual. */
tmamg_status tmamg_solve_shifted(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* sigma, double tol,
                                 tmamg_info* info);

/* The even-odd reduced system D_hat(mu_r) x_r = b_r on the even sites
 * (x + y + z + t even), D_hat = D_ee - D_eo D_oo^-1 D_oe: the operator the
 * paper's simulations use (Sec. 1.2).  Solved through the full operator
 * (D [x_e; x_o] = [b_e; 0] gives D_hat x_e = b_e) with the FP64 residual of
 * the reduced system checked by the Schur operator and corrected while
 * above tol.  b, x: device canonical spinors [nrhs]; odd entries of b are
 * ignored, odd entries of x are set to 0; mu_rhs as for tmamg_solve;
 * info.true_rel_resid is the reduced system's ||b_e - D_hat x_e|| / ||b_e||.
 * Assumes the site-diagonal term's Hermitian part is positive definite (as
 * TMAMG_OP_SCHUR64). */
tmamg_status tmamg_solve_eo(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                            tmamg_info* info);

/* Shifted systems of one source, (D D^dag + sigma_k) x_k = b for k < nshift,
 * with the first-order initial guesses of Sec. 3, Eq. (6): the shifted
 * inverse expanded in the shift, (Q +- i delta)^-1 ~ Q^-1 -+ i delta Q^-2,
 * with Q = Gamma5 D(0) + i mu_b around the smallest shift's twisted mass
 * mu_b = sqrt(mu^2 + sigma_min), applied to both solves of each shift (the
 * base shift takes four solves, the others start from the guesses; a guess
 * worse than zero is dropped).  Each shifted system's own FP64 residual is
 * then corrected as in tmamg_solve_shifted.  b: device canonical spinor [1];
 * x: device canonical [nshift]; sigma: host [nshift], >= 0.  The guess pays
 * when the shifts are close (delta small against the low modes). */
tmamg_status tmamg_solve_multishift(tmamg_ctx* ctx, const void* b, void* x, int nshift, const double* sigma,
                                    double tol, tmamg_info* info);

/* Non-degenerate doublet (Sec. 1.1, Eq. 2): solve
 *   D_ND(mubar, epsbar) x = b,  D_ND = [[D(mubar), -epsbar], [-epsbar, D(-mubar)]]
 * with the hierarchy built at setup (P_ND = P x I_2: each flavour's
 * multigrid cycle at its own twisted mass +-mubar preconditions one flexible
 * Krylov space over both flavours; the coupling enters the outer operator).
 * b, x: device, canonical spinors [2] (flavour-major, the flavours' fields
 * back to back).  Stops when ||b - D_ND x|| / ||b|| <= tol over both
 * flavours together (FP64 true residual). */
tmamg_status tmamg_solve_nd(tmamg_ctx* ctx, const void* b, void* x, double mubar, double epsbar, double tol,
                            tmamg_info* info);

/* Pseudofermion action S_f = phi^dag (D D^dag)^-1 phi at the setup mu and
 * its force F_mu(x) = sum_a (dS/dw^a) T^a for U -> exp(w) U, T^a = i lambda^a/2
 * (dS/dt = -2 sum tr(F w)); F is traceless anti-Hermitian.  The HMC force
 * of Sec. 1.2 (its solves use the DD-alpha-AMG of Sec. 1.1 to tol; the
 * paper's MD forces use 1e-9) and Sec. 2: Y = D^-1 phi, X = (D^dag)^-1 Y,
 * then the adjoint of the hopping and clover terms on (X, Y).
 * phi: device spinor [1]; F: device [4][T][Z][Y][X][3][3]; S: host. */
tmamg_status tmamg_force(tmamg_ctx* ctx, const void* phi, void* F, double* S, double tol, tmamg_info* info);

/* tmamg_force at twisted mass mu instead of the setup's (the hierarchy
 * serves every mu, Sec. 1.1): the monomials of Sec. 2, Eq. (3), each at
 * its own shifted mass. */
tmamg_status tmamg_force_at(tmamg_ctx* ctx, const void* phi, double mu, void* F, double* S, double tol,
                            tmamg_info* info);

/* Molecular dynamics of the HMC of Sec. 2 (the nested integrator's
 * updates; the gauge action on its innermost time scale).  Canonical
 * complex128 fields [4][T][Z][Y][X][3][3] on the device; the gauge field is
 * periodic.  gauge_force: S = beta sum_{x, mu<nu} (1 - Re tr P_{mu nu}(x)/3)
 * (host) and its force F = sum_a (dS/dw^a) T^a for U -> exp(w) U (the
 * convention of tmamg_force).  md_update_links: U <- exp(eps P) U per link
 * (P traceless anti-Hermitian).  md_update_momenta: P <- P + coef F.
 * md_kinetic: K = sum |P_ij|^2 = 1/2 sum_a (p^a)^2 (host). */
tmamg_status tmamg_gauge_force(tmamg_ctx* ctx, const void* U, double beta, void* F, double* S);
tmamg_status tmamg_md_update_links(tmamg_ctx* ctx, void* U, const void* P, double eps);
tmamg_status tmamg_md_update_momenta(tmamg_ctx* ctx, void* P, const void* F, double coef);
tmamg_status tmamg_md_kinetic(tmamg_ctx* ctx, const void* P, double* K);

/* The force of tmamg_force (Sec. 1.2) for given X = (D D^dag)^-1 phi and
 * Y = D^dag X (device canonical spinors), without solves: F from the
 * hopping and clover derivatives.  F: device [4][T][Z][Y][X][3][3]. */
tmamg_status tmamg_force_from_fields(tmamg_ctx* ctx, const void* X, const void* Y, void* F);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the force
 * of tmamg_force_from_fields with every intermediate field in a static
 * device scratch array of 160 MiB per GPU, held from the first context on
 * that GPU until the process ends.  It needs 78 complex doubles per site
 * (at most 134,432 sites: a 16^3 x 32 lattice fits; larger lattices get
 * TMAMG_EINVAL) and allocates nothing.  Every call on one GPU uses that
 * GPU's single array: calls that overlap on one GPU (several contexts,
 * threads or streams) race.  Same arguments and result as
 * tmamg_force_from_fields. */
tmamg_status tmamg_force_from_fields_noalloc(tmamg_ctx* ctx, const void* X, const void* Y, void* F);

/* Link gradient of S_f for automatic differentiation (Sec. 1.2 force, as
 * a gradient): G_mu(x) = 2 scale F_mu(x) U_mu(x), with F a force from
 * tmamg_force at the context's current links U.  For every perturbation
 * U -> exp(X) U with X traceless anti-Hermitian, the first-order change of
 * scale * S_f is Re sum conj(G) (X U): G is the complex gradient
 * dS/dRe U + i dS/dIm U (PyTorch's convention) on the directions tangent
 * to SU(3); its component normal to SU(3) is not computed.  F, G: device
 * [4][T][Z][Y][X][3][3] complex128 (may not alias); scale: host. */
tmamg_status tmamg_force_link_gradient(tmamg_ctx* ctx, const void* F, void* G, double scale);

/* Operator hook for tests: the single steps of the method of Sec. 1.1
 * (operator, transfers P and P^dag, Galerkin D_c, SAP, the cycle of
 * Eq. (1), the coarsest solve).  op: one of TMAMG_OP_*; level: 0 fine, 1,
 * 2.  in/out: device, canonical fields of that level, nrhs of them (may not
 * alias); mu_rhs host [nrhs] or NULL (setup mu). */
enum {
  TMAMG_OP_D64 = 0,       /* fine D(mu) in FP64 */
  TMAMG_OP_D32 = 1,       /* fine D(mu) in FP32 (rounded in/out) */
  TMAMG_OP_PROLONG = 2,   /* level -> level-1: out = P in (in: coarse field of level `level`) */
  TMAMG_OP_RESTRICT = 3,  /* level -> level+1: out = P^dag in */
  TMAMG_OP_DC = 4,        /* coarse D_c(mu) on level 1 or 2 */
  TMAMG_OP_SAP = 5,       /* k SAP sweeps from zero on level 0 or 1: out ~ D^-1 in */
  TMAMG_OP_PREC = 6,      /* one multigrid cycle B_MG on level 0 or 1 */
  TMAMG_OP_COARSEST = 7,  /* coarsest-level GMRES from zero (coarsest_iters, coarsest_tol) on
                             level nlevels-1: out ~ D_c^-1 in */
  TMAMG_OP_SCHUR64 = 8,   /* even-odd reduced fine operator in FP64 (Sec. 1.2 even-odd
                             preconditioning): out = (D_ee - D_eo D_oo^-1 D_oe) in on the
                             sites with x+y+z+t even; odd entries of in are ignored, odd
                             entries of out are 0.  Level 0.  Assumes the Hermitian part
                             of the site-diagonal term is positive definite (m0 + 4 above
                             the clover term's spectral radius) */
  TMAMG_OP_SCHUR32 = 9,   /* the same in FP32 (rounded in/out) */
  TMAMG_OP_DDAG64 = 10,   /* fine D(mu)^dag = Gamma5 D(-mu) Gamma5 in FP64 (Sec. 1.1) */
  TMAMG_OP_DDAG32 = 11,   /* the same in FP32 (rounded in/out) */
  TMAMG_OP_DCND = 12,     /* doublet coarse operator D_ND,c = P_ND^dag D_ND P_ND (Sec. 1.1,
                             Eq. (2), P_ND = P x I_2) on level 1 or 2: nrhs = 2 (the two
                             flavours' coarse fields), mu_rhs = {mubar, epsbar} (required) */
  TMAMG_OP_SAPND = 13     /* the doublet's fine SAP (k sweeps from zero, level 0) on the
                             coupled block operator D_ND restricted to the blocks: nrhs = 2,
                             mu_rhs = {mubar, epsbar}.  Mixed precision couples the
                             flavours in the block solves; FP64 smooths each flavour alone */
};
tmamg_status tmamg_apply(tmamg_ctx* ctx, int op, int level, const void* in, void* out, int nrhs,
                         const double* mu_rhs);

/* Test hook for failure paths (no passage of the paper): what = 0 marks a timed-out barrier wait in the
 * persistent coarse kernels' status word, as a real timeout would; the next
 * solve then returns TMAMG_EHIP and the context falls back to the generic
 * coarse kernels.  Needs a setup with two or more levels. */
tmamg_status tmamg_debug_inject(tmamg_ctx* ctx, int what);

/* Test hooks for parity of the setup's P and D_c (Sec. 1.1: P from the
 * test vectors, D_c = P^dag D P).  set_test_vectors: the next setup starts from these N_v
 * vectors of level `level` (device, canonical level fields) instead of noise.
 * export: what = 0 copies P of coarsening `level` (N_v canonical fields of
 * the finer level, complex128) to out; what = 1 copies D_c of level
 * `level` (1 or 2) as complex128 [Vc][9][d][d] with blocks (self, +x, -x,
 * +y, -y, +z, -z, +t, -t), each [column][row]. */
tmamg_status tmamg_debug_set_test_vectors(tmamg_ctx* ctx, int level, const void* v);
tmamg_status tmamg_debug_export(tmamg_ctx* ctx, int what, int level, void* out);

/* Measurement (no passage of the paper): kernel timing; launches kernel `kernel` `reps` times on
 * internal buffers of nrhs right-hand sides (random contents) between two
 * HIP events on the context's stream and stores the mean milliseconds per
 * launch in *avg_ms (host).  Kernels: TMAMG_K_*. Needs a completed setup
 * for the multigrid kernels. */
enum {
  TMAMG_K_DSLASH32 = 0,   /* fine stencil, FP32 */
  TMAMG_K_DSLASH64 = 1,   /* fine stencil, FP64 */
  TMAMG_K_SAP0 = 2,       /* fine SAP, one colour (hierarchy precision) */
  TMAMG_K_RESTRICT0 = 3,  /* fine -> level 1 */
  TMAMG_K_PROLONG0 = 4,   /* level 1 -> fine */
  TMAMG_K_DC1 = 5,        /* coarse operator, level 1 */
  TMAMG_K_DC2 = 6,        /* coarse operator, level 2 */
  TMAMG_K_SAP1 = 7,       /* coarse SAP on level 1, one sweep (both colours) */
  TMAMG_K_COPY = 8,       /* plain device copy of 512 MiB (counter calibration) */
  TMAMG_K_SCHUR32 = 9     /* even-odd reduced fine operator, FP32 (both half passes) */
};
tmamg_status tmamg_time_kernel(tmamg_ctx* ctx, int kernel, int nrhs, int reps, double* avg_ms);

/* Kernel variant tuning (measurement and plumbing; the paper has nothing to
 * say about it).  Some steps have two correct kernels for one shape; the
 * launcher picks one by a built-in rule unless the process-wide variant
 * table holds an entry for its family and shape key (a, b, nrhs):
 *   TMAMG_TUNE_COARSE_APPLY  a = dof per coarse site, b = coarse sites;
 *                            0 vector ALU, 1 matrix cores (16 RHS tiles)
 *   TMAMG_TUNE_SAP1          level-1 SAP, same key; 0 vector ALU, 1 matrix
 *                            cores, 2 matrix cores with a register budget for
 *                            four workgroups per CU, 3 matrix cores with one
 *                            workgroup per SAP block (blocks of at most 16
 *                            sites, d <= 48; the colour in one launch)
 *   TMAMG_TUNE_RESTRICT0,
 *   TMAMG_TUNE_PROLONG0      a = N_v, b = fine sites; 0 vector ALU, 1 matrix cores
 *   TMAMG_TUNE_SAP0          fine SAP, a = block sites, b = fine sites;
 *                            register budget for 0 one / 1 three workgroups per CU,
 *                            one right-hand side per workgroup; 2: two right-hand
 *                            sides per workgroup (lane pairs on one site share every
 *                            link and clover load)
 * A variant a launcher cannot run for its precision, storage or shape is
 * ignored (the rule applies).  Every variant computes the same operation;
 * results differ only by rounding (SAP0 variants not at all).  The table
 * is shared by all contexts of the process and is not locked against
 * concurrent tuning from several threads. */
enum {
  TMAMG_TUNE_COARSE_APPLY = 0,
  TMAMG_TUNE_SAP1 = 1,
  TMAMG_TUNE_RESTRICT0 = 2,
  TMAMG_TUNE_PROLONG0 = 3,
  TMAMG_TUNE_SAP0 = 4
};
/* Measurement and plumbing: the autotuner.  For every right-hand-side
 * count nrhs_list[0..n) (host, each 1..64) and every family with two
 * variants for this context's hierarchy, times each variant over `reps`
 * launches (HIP events, as tmamg_time_kernel) and stores the faster in the
 * table.  json_path: if not NULL, the whole table is written there as JSON
 * (entries with the measured milliseconds of each variant).  Needs a
 * completed setup. */
tmamg_status tmamg_autotune(tmamg_ctx* ctx, const int* nrhs_list, int n, int reps, const char* json_path);
/* Plumbing: add the entries of a file written by tmamg_autotune or
 * tmamg_tune_save (same keys are replaced); *n_entries (may be NULL) =
 * entries read.
 * TMAMG_EINVAL if the file is unreadable or malformed (nothing is added). */
tmamg_status tmamg_tune_load(const char* json_path, int* n_entries);
tmamg_status tmamg_tune_save(const char* json_path);
/* Plumbing: set one entry (variant -1 removes it; TMAMG_EINVAL beyond the
 * family's variants); read one (-1: none). */
tmamg_status tmamg_tune_set(int family, long a, long b, long nrhs, int variant);
int tmamg_tune_get(int family, long a, long b, long nrhs);
int tmamg_tune_entries(void);
void tmamg_tune_clear(void);

/* Plumbing: sizes of level `level`: sites and dof per site (fine: 12;
 * coarse: 2 N_v, Sec. 1.1). */
tmamg_status tmamg_level_info(const tmamg_ctx* ctx, int level, long* sites, int* dof);

/* Plumbing: release the context and every buffer it owns (through the
 * allocator given at creation).  NULL is ignored. */
void tmamg_destroy(tmamg_ctx* ctx);

/* Plumbing: message for the last non-OK status of the calling thread. */
const char* tmamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TMAMG_H */
