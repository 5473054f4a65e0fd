// Host-side types of the solver library.
#pragma once

#include "kernels.h"
#include "tmamg.h"

#include <functional>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

struct TmError {
  tmamg_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                                  \
  do {                                                                                             \
    hipError_t e_ = (x);                                                                           \
    if (e_ != hipSuccess)                                                                          \
      throw TmError{TMAMG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

extern thread_local std::string g_last_error;

// Where a context's device buffers come from: hipMalloc/hipFree, or the
// pair of callbacks the caller installed at creation (for example a
// framework's caching allocator).  g_alloc names the allocator of the API
// call in progress on this thread (null outside calls: hipMalloc); every
// buffer remembers the allocator that produced it and is released with it.
struct DevAlloc {
  tmamg_alloc_fn alloc = nullptr;
  tmamg_free_fn free = nullptr;
  void* user = nullptr;
  hipStream_t st = nullptr;
};
extern thread_local const DevAlloc* g_alloc;
struct AllocScope {
  const DevAlloc* saved;
  explicit AllocScope(const DevAlloc* a) : saved(g_alloc) { g_alloc = a; }
  ~AllocScope() { g_alloc = saved; }
};

template <typename X>
struct DevArr {
  X* p = nullptr;
  size_t n = 0;
  int count = 0;   // optional element count used by callers (e.g. block lists)
  DevAlloc from{};
  DevArr() = default;
  DevArr(const DevArr&) = delete;
  DevArr& operator=(const DevArr&) = delete;
  ~DevArr() { release(); }
  void alloc(size_t cnt) {
    if (cnt == n && p) return;
    release();
    if (cnt == 0) return;
    const size_t bytes = cnt * sizeof(X);
    if (g_alloc && g_alloc->alloc) {
      from = *g_alloc;
      p = static_cast<X*>(from.alloc(bytes, from.st, from.user));
      if (!p) {
        from = DevAlloc{};
        throw TmError{TMAMG_ENOMEM, "the caller's allocator refused " + std::to_string(bytes) + " bytes"};
      }
    } else {
      from = DevAlloc{};
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        throw TmError{TMAMG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
      }
    }
    n = cnt;
  }
  void release() {
    if (p) {
      if (from.free) from.free(p, from.st, from.user);
      else (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    from = DevAlloc{};
  }
  size_t bytes() const { return n * sizeof(X); }
};

template <typename T>
using OpFn = std::function<void(const cplx<T>*, cplx<T>*)>;

template <typename T>
struct Krylov {
  int m = 0, cap = 0, NB = 1;
  long n = 0;
  bool flex = false;
  DevArr<cplx<T>> V, Z, w;
  DevArr<double> H, cs, sn, g, c1, c2, nrm, inv, beta0, tol, y, partial;
  DevArr<int> active, kdone, status, reorth;
  void ensure(long n_, int m_, int nrhs, bool flex_, hipStream_t st);
  KrylovDev dev() const;
};

template <typename T>
int krylov_cycle(Krylov<T>& K, const OpFn<T>& A, const OpFn<T>* M, const cplx<T>* r0, cplx<T>* x, int nrhs,
                 int maxit, double reltol, const double* abstol, bool host_check, int* host_flags, hipStream_t st);

struct Ctx;

// Phase timing with HIP events on the library stream, enabled by the
// environment variable TMAMG_TIMING=1; a summary line goes to stderr after
// each setup and solve.
struct PhaseTimer {
  enum { FINE_SAP, FINE_TRANSFER, L1_SOLVE, L1_SAP, COARSEST, OUTER_OP, SETUP_BUILD, NPH };
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int ph; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  hipEvent_t begin(hipStream_t st) {
    if (!on) return nullptr;
    hipEvent_t a = ev();
    HIPCHK(hipEventRecord(a, st));
    return a;
  }
  void end(int ph, hipEvent_t a, hipStream_t st) {
    if (!on) return;
    hipEvent_t b = ev();
    HIPCHK(hipEventRecord(b, st));
    recs.push_back({ph, a, b});
  }
  void report(const char* tag, hipStream_t st, const std::string& extra = "");
  ~PhaseTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct HierBase {
  virtual ~HierBase() {}
  virtual void setup(double mu) = 0;
  virtual void setup_iteration() = 0;
  virtual void rebuild() = 0;
  // memory plan: drop the setup's work buffers (and the fine test vectors
  // unless the parameters keep them); has_test_vectors() tells whether
  // setup updates are still possible
  virtual void release_setup_workspace() {}
  virtual bool has_test_vectors() const { return true; }
  virtual void ensure(int nrhs) = 0;
  virtual bool is_double() const = 0;
  // typed entry points; only the matching precision is implemented
  virtual void precond_d(const cplx<double>*, cplx<double>*, int, const double*) { throw TmError{TMAMG_ESTATE, "precision"}; }
  virtual void precond_f(const cplx<float>*, cplx<float>*, int, const double*) { throw TmError{TMAMG_ESTATE, "precision"}; }
  // test hook on internal buffers of the hierarchy precision
  virtual void test_op(int op, int level, const void* in, void* out, int nrhs, const double* mu) = 0;
  virtual void export_P(int level, cplx<double>* out) = 0;
  virtual void export_Dc(int level, cplx<double>* out) = 0;
  virtual double time_kernel(int kernel, int nrhs, int reps) = 0;
  virtual void autotune(int nrhs, int reps) = 0;
  // counters of the coarse solves since the last call (and reset them)
  struct Counters {
    long l2 = 0, coarsest = 0;
    int coarsest_calls = 0, reorth = 0, timeouts = 0;
  };
  virtual Counters take_counters() { return Counters{}; }
  // persistent coarse kernels: mark a barrier timeout as if one had
  // happened (failure-path tests), and stop using them after one
  virtual void flag_barrier_timeout() {}
  virtual void disable_persistent() {}
  long stats_l2 = 0, stats_coarsest = 0;
  PhaseTimer* timer = nullptr;
  // non-zero while a doublet (two flavours as a pair of right-hand sides)
  // is solved: the coarse operators carry the flavour coupling -epsbar
  double nd_eps = 0.0;
};

template <typename T, typename S>
struct Hier : HierBase {
  using SPair = typename Store<S>::pair;
  Ctx* c;
  int nlev = 1;
  FineOp<T> fop;
  int nv0 = 0, nv1 = 0, d1 = 0, d2 = 0;
  CoarseGeom g1{}, g2{};
  DevArr<int> blist0[2], blist1[2];
  DevArr<cplx<T>> tv0, tv1, tvtmp, tmp1;
  DevArr<cplx<T>> gal_ws;   // fine Galerkin workspace (columns of D P per receiving aggregate)
  DevArr<SPair> P0, P1, Dc1, Dc2;
  DevArr<cplx<double>> P64;
  DevArr<cplx<T>> rc1, ec1, rc2, ec2;
  Krylov<T> K1, K2;
  Krylov<T> KN1, KN2;   // doublet: one Krylov space over both flavours per coarse level
  DevArr<double> red_partial, red_out, red_inv, mu_setup;
  // fused coarse SAP: residual/product vectors and per-site partial sums,
  // two slots each; coarsest-GMRES scalars, flags and barrier counters
  DevArr<cplx<T>> sap_rho[2], sap_q[2];
  DevArr<double> sap_part[2], cg_dws;
  DevArr<int> cg_iws;
  int cap = 0;
  bool use_coop = true;
  // captured intermediate-level solves (rc1 -> ec1), one per right-hand-side
  // count and twisted-mass array; `calls` counts eager uses before capture
  struct GraphEntry { int nrhs; const double* mu; int calls; hipGraphExec_t exec; long l2_steps, coarsest_steps; };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_st = nullptr;
  bool capturing = false;

  explicit Hier(Ctx* c_);
  ~Hier() override;
  void drop_graphs();
  bool coarse_solve_graph(int nrhs, const double* mu);
  void build_colours(const int nb[4], DevArr<int> out[2]);
  void ensure(int nrhs) override;
  Counters take_counters() override;
  void flag_barrier_timeout() override;
  void disable_persistent() override { use_coop = false; drop_graphs(); }
  void dc_apply(int level, const cplx<T>* in, cplx<T>* out, int nrhs, const double* mu);
  void sap(int level, const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu, int sweeps);
  void sap_level1(const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu, int sweeps);
  void precond(int level, const cplx<T>* v, cplx<T>* z, int nrhs, const double* mu);
  void coarse_solve(int level, const cplx<T>* rhs, cplx<T>* sol, int nrhs, const double* mu);
  void coarse_solve_nd(int level, const cplx<T>* rhs, cplx<T>* sol, const double* mu);
  void normalize(cplx<T>* v, long n, int nrhs);
  void build(int l);
  void build_inner(int l);
  void galerkin_only(int l);
  void setup(double mu) override;
  void smooth_vectors(int l);
  void setup_iteration() override;
  void rebuild() override;
  void release_setup_workspace() override;
  bool has_test_vectors() const override { return nlev < 2 || tv0.p != nullptr; }
  void setup_workspace();
  int chunk(int l) const;
  bool is_double() const override { return std::is_same<T, double>::value; }
  void precond_d(const cplx<double>* v, cplx<double>* z, int nrhs, const double* mu) override;
  void precond_f(const cplx<float>* v, cplx<float>* z, int nrhs, const double* mu) override;
  void test_op(int op, int level, const void* in, void* out, int nrhs, const double* mu) override;
  void export_P(int level, cplx<double>* out) override;
  void export_Dc(int level, cplx<double>* out) override;
  double time_kernel(int kernel, int nrhs, int reps) override;
  void autotune(int nrhs, int reps) override;
};

struct Ctx {
  tmamg_lattice lat{};
  tmamg_params par{};
  hipStream_t st = nullptr;
  FineGeom fg{};
  DevArr<cplx<double>> links64;
  DevArr<cplx<float>> links32;
  DevArr<double> clov64;
  DevArr<float> clov32;
  double kappa = 0, m0 = 0, csw = 0, mu = 0;
  bool have_links = false, have_setup = false;
  std::unique_ptr<HierBase> hier;
  DevArr<cplx<double>> inject0, inject1;
  // solve workspace
  Krylov<double> K64;
  Krylov<float> K32;
  Krylov<double> KN64;   // doublet solves: one Krylov space over both flavours
  Krylov<float> KN32;
  DevArr<cplx<double>> b64, x64, r64, t64;
  DevArr<cplx<float>> r32, e32;
  DevArr<double> mu_dev, abstol_dev, red_partial, red_out;
  // the twisted masses of the current solve (host), and the device copy
  // for the right-hand sides of a compacted cycle
  std::vector<double> mu_now;
  DevArr<double> mu_cdev;
  DevArr<cplx<double>> c64;   // FP64 corrections of a compacted cycle (allocated on first use)
  int* host_flags = nullptr;
  PhaseTimer timer;
  double t_setup = 0;
  int cap = 0;

  DevAlloc dalloc{};   // where the context's device buffers come from
  // shifted systems: the original right-hand sides, the accumulated solution
  DevArr<cplx<double>> sh_b, sh_x;

  Ctx(const tmamg_lattice& l, const tmamg_params& p, hipStream_t s, const tmamg_allocator* a);
  ~Ctx();
  FineOp<double> op64() const { FineOp<double> o; o.g = fg; o.links = links64.p; o.clover = clov64.p; return o; }
  FineOp<float> op32() const { FineOp<float> o; o.g = fg; o.links = links32.p; o.clover = clov32.p; return o; }
  void load_links(const cplx<double>* U);
  void setup(const cplx<double>* U, double kappa, double csw, double mu);
  void setup_update(const cplx<double>* U, int iters);
  void ensure(int nrhs);
  std::vector<double> norms(const cplx<double>* v, int nrhs);
  tmamg_status solve_core(int nrhs, const double* mu_host, double tol, tmamg_info* info,
                          const double* eps_nd = nullptr, bool guess = false);
  tmamg_status finish(tmamg_info& loc, tmamg_status s);
  HierBase::Counters drain_counters();
  tmamg_status solve_nd(const cplx<double>* b, cplx<double>* x, double mubar, double epsbar, double tol,
                        tmamg_info* info);
  tmamg_status solve(const cplx<double>* b, cplx<double>* x, int nrhs, const double* mu_host, double tol,
                     tmamg_info* info, bool guess = false);
  tmamg_status solve_shifted(const cplx<double>* b, cplx<double>* x, int nrhs, const double* sigma, double tol,
                             tmamg_info* info);
  tmamg_status solve_multishift(const cplx<double>* b, cplx<double>* x, int nshift, const double* sigma, double tol,
                                tmamg_info* info);
  tmamg_status solve_eo(const cplx<double>* b, cplx<double>* x, int nrhs, const double* mu_host, double tol,
                        tmamg_info* info);
  // FP64 residuals r_k = b_k - (D D^dag + sigma_k) x_k (internal layout) and their relative norms
  std::vector<double> shifted_residual(const cplx<double>* b, const cplx<double>* x, cplx<double>* r, int nrhs,
                                       const std::vector<double>& mup, const std::vector<double>& bn);
  DevArr<cplx<double>> ms_base;   // multishift: the base shift's four fields
  tmamg_status force(const cplx<double>* phi, cplx<double>* F, double* S, double tol, tmamg_info* info,
                     const double* mu_force = nullptr);
  void force_from_fields(const cplx<double>* X, const cplx<double>* Y, cplx<double>* F);
  void force_from_fields_ws(const cplx<double>* X, const cplx<double>* Y, cplx<double>* F, cplx<double>* ws);
  void* scratch = nullptr;   // this device's static scratch array (allocation-free entry point)
  void force_link_gradient(const cplx<double>* F, cplx<double>* G, double scale);
  void apply(int op, int level, const cplx<double>* in, cplx<double>* out, int nrhs, const double* mu_host);
  void upload_mu(int nrhs, const double* mu_host);
  double time_kernel(int kernel, int nrhs, int reps);
  void autotune(const int* nrhs_list, int n, int reps);
};

// mean milliseconds per call of f over reps calls, HIP events on st
template <typename F>
double time_launches(hipStream_t st, int reps, F&& f) {
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  f();   // warm
  HIPCHK(hipEventRecord(a, st));
  for (int i = 0; i < reps; ++i) f();
  HIPCHK(hipEventRecord(b, st));
  HIPCHK(hipEventSynchronize(b));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// force kernels (K13-K15)
// xi_ws: workspace of 54 complex doubles per site for the clover part, or
// null (then it is allocated for the call)
void launch_force(const FineOp<double>& op, double csw, const cplx<double>* X, const cplx<double>* Y,
                  cplx<double>* F_canon, hipStream_t st, cplx<double>* xi_ws = nullptr);
void launch_link_gradient(const FineOp<double>& op, int antiperiodic, const cplx<double>* F_canon,
                          cplx<double>* G_canon, double scale, hipStream_t st);

// molecular-dynamics pieces (md.hip), canonical layouts
double md_gauge_force(const tmamg_lattice& lat, const cplx<double>* U, double beta, cplx<double>* F, hipStream_t st);
void md_update_links(const tmamg_lattice& lat, cplx<double>* U, const cplx<double>* P, double eps, hipStream_t st);
void md_update_momenta(const tmamg_lattice& lat, cplx<double>* P, const cplx<double>* F, double c, hipStream_t st);
double md_kinetic(const tmamg_lattice& lat, const cplx<double>* P, hipStream_t st);
