// Host orchestration of the DD-alpha-AMG solver (Sec. 1.1 of arXiv:1710.06198):
// the multigrid hierarchy, its cycle (Eq. (1): coarse-grid correction, then
// k SAP sweeps), the adaptive setup, the flexible Krylov drivers, and the
// mixed-precision defect correction around FP32 cycles.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

thread_local std::string g_last_error;
thread_local const DevAlloc* g_alloc = nullptr;

// ------------------------------------------------------------------ small kernels
__global__ void k_rsqrt(const double* in, double* out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] > 0 ? 1.0 / sqrt(in[i]) : 0.0;
}
__global__ void k_fill_double(double* p, double v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

struct DoubleChunk {
  double v[32];
};
__global__ void k_set_doubles(double* p, DoubleChunk c, int n) {
  const int i = threadIdx.x;
  if (i < n) p[i] = c.v[i];
}
void launch_set_doubles(double* dst, const double* vals, int n, hipStream_t st) {
  for (int o = 0; o < n; o += 32) {
    DoubleChunk c{};
    const int k = std::min(32, n - o);
    for (int i = 0; i < k; ++i) c.v[i] = vals[o + i];
    hipLaunchKernelGGL(k_set_doubles, dim3(1), dim3(32), 0, st, dst + o, c, k);
  }
}

void PhaseTimer::report(const char* tag, hipStream_t st, const std::string& extra) {
  if (!on) return;
  HIPCHK(hipStreamSynchronize(st));
  double t[NPH] = {0};
  for (const Rec& r : recs) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    t[r.ph] += ms;
  }
  static const char* names[NPH] = {"fine_sap", "fine_transfer", "level1_solve", "level1_sap", "coarsest",
                                   "outer_operator", "setup_build"};
  fprintf(stderr, "[tmamg timing] %s", tag);
  for (int i = 0; i < NPH; ++i) fprintf(stderr, " %s=%.2fms", names[i], t[i]);
  fprintf(stderr, "%s\n", extra.c_str());
  recs.clear();
  used = 0;
}

// ------------------------------------------------------------------ Krylov driver
template <typename T>
void Krylov<T>::ensure(long n_, int m_, int nrhs, bool flex_, hipStream_t st) {
  if (n == n_ && m >= m_ && cap >= nrhs && (flex || !flex_)) return;
  n = n_;
  m = std::max(m, m_);
  cap = std::max(cap, nrhs);
  flex = flex || flex_;
  NB = reduce_blocks(n);
  V.alloc((size_t)(m + 1) * cap * n);
  if (flex) Z.alloc((size_t)m * cap * n);
  w.alloc((size_t)cap * n);
  H.alloc(2 * (size_t)cap * (m + 1) * m);
  cs.alloc(2 * (size_t)cap * m);
  sn.alloc(2 * (size_t)cap * m);
  g.alloc(2 * (size_t)cap * (m + 1));
  c1.alloc(2 * (size_t)cap * (m + 1));
  c2.alloc(2 * (size_t)cap * (m + 1));
  nrm.alloc(cap);
  inv.alloc(cap);
  beta0.alloc(cap);
  tol.alloc(cap);
  y.alloc(2 * (size_t)cap * m);
  partial.alloc(2 * (size_t)cap * (m + 1) * NB);
  active.alloc(cap);
  kdone.alloc(cap);
  status.alloc(cap);
  reorth.alloc(cap);
  launch_fill_zero(V.p, V.bytes(), st);
  if (flex) launch_fill_zero(Z.p, Z.bytes(), st);
  launch_fill_zero(w.p, w.bytes(), st);
  launch_fill_zero(active.p, active.bytes(), st);
  launch_fill_zero(kdone.p, kdone.bytes(), st);
  launch_fill_zero(inv.p, inv.bytes(), st);
}

template <typename T>
KrylovDev Krylov<T>::dev() const {
  KrylovDev k;
  k.m = m;
  k.H = H.p; k.cs = cs.p; k.sn = sn.p; k.g = g.p; k.c1 = c1.p; k.c2 = c2.p;
  k.nrm = nrm.p; k.inv = inv.p; k.beta0 = beta0.p; k.tol = tol.p; k.y = y.p;
  k.active = active.p; k.kdone = kdone.p; k.status = status.p; k.reorth = reorth.p;
  return k;
}

// One (F)GMRES cycle of at most maxit steps for A e = r0, accumulating into x:
// x += Z y (flexible) or V y.  Per-RHS predication: a right-hand side stops
// contributing once its implicit residual meets its target.  With
// host_check the host reads the active flags after every step and ends the
// cycle early; without it the launch schedule is fixed.
template <typename T>
int krylov_cycle(Krylov<T>& K, const OpFn<T>& A, const OpFn<T>* M, const cplx<T>* r0, cplx<T>* x, int nrhs,
                 int maxit, double reltol, const double* abstol, bool host_check, int* host_flags, hipStream_t st) {
  const long n = K.n;
  const long vs = (long)nrhs * n;
  KrylovDev kd = K.dev();
  const int NB = K.NB;
  maxit = std::min(maxit, K.m);
  launch_norm2(r0, n, nrhs, K.partial.p, NB, nullptr, st);
  launch_finalize_real(K.partial.p, nrhs, NB, kd.nrm, st);
  launch_krylov_start(kd, reltol, abstol, nrhs, st);
  launch_scale_dev(r0, K.V.p, kd.inv, n, nrhs, nullptr, st);
  int done = 0;
  if (host_check) {
    HIPCHK(hipMemcpyAsync(host_flags, kd.active, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool any = false;
    for (int r = 0; r < nrhs; ++r) any |= host_flags[r] != 0;
    if (!any) return 0;
  }
  for (int j = 0; j < maxit; ++j) {
    cplx<T>* vj = K.V.p + (long)j * vs;
    cplx<T>* zj = vj;
    if (M) {
      zj = K.Z.p + (long)j * vs;
      (*M)(vj, zj);
    }
    // the new vector is formed in its own basis slot, so the first pass's
    // dot products also give |w|^2 (the last of j + 2); the second pass
    // runs only where the first cancelled more than a factor 10 of |w|
    cplx<T>* wj = K.V.p + (long)(j + 1) * vs;
    A(zj, wj);
    launch_multidot(K.V.p, vs, j + 2, wj, n, nrhs, K.partial.p, NB, kd.active, st);
    launch_finalize(K.partial.p, nrhs * (j + 2), j + 2, NB, kd.c1, K.m + 1, st);
    launch_multiaxpy(wj, K.V.p, vs, j + 1, kd.c1, K.m + 1, n, nrhs, -1.0, kd.active, st);
    launch_cgs_decide(kd, j, nrhs, 0.01, st);
    launch_multidot(K.V.p, vs, j + 1, wj, n, nrhs, K.partial.p, NB, kd.reorth, st);
    launch_finalize(K.partial.p, nrhs * (j + 1), j + 1, NB, kd.c2, K.m + 1, st, kd.reorth);
    launch_multiaxpy(wj, K.V.p, vs, j + 1, kd.c2, K.m + 1, n, nrhs, -1.0, kd.reorth, st);
    launch_norm2(wj, n, nrhs, K.partial.p, NB, kd.active, st);
    launch_finalize_real(K.partial.p, nrhs, NB, kd.nrm, st);
    launch_krylov_step(kd, j, nrhs, st);
    if (j + 1 < maxit) launch_scale_dev(wj, wj, kd.inv, n, nrhs, nullptr, st);
    done = j + 1;
    if (host_check) {
      HIPCHK(hipMemcpyAsync(host_flags, kd.active, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool any = false;
      for (int r = 0; r < nrhs; ++r) any |= host_flags[r] != 0;
      if (!any) break;
    }
  }
  launch_krylov_solve_y(kd, nrhs, st);
  launch_krylov_update(x, M ? K.Z.p : K.V.p, vs, kd, n, nrhs, st);
  return done;
}

// ------------------------------------------------------------------ hierarchy
template <typename T, typename S>
Hier<T, S>::Hier(Ctx* c_) : c(c_) {
  const tmamg_params& p = c->par;
  nlev = p.nlevels;
  fop.g = c->fg;
  if constexpr (std::is_same<T, double>::value) {
    fop.links = c->links64.p;
    fop.clover = c->clov64.p;
  } else {
    fop.links = c->links32.p;
    fop.clover = c->clov32.p;
  }
  // fine SAP colour lists (blocks = aggregates of the fine ordering)
  build_colours(c->fg.NB, blist0);
  if (nlev >= 2) {
    nv0 = p.nv[0];
    d1 = 2 * nv0;
    g1.V = 1;
    for (int m = 0; m < 4; ++m) { g1.L[m] = c->fg.NB[m]; g1.V *= g1.L[m]; }
  }
  if (nlev >= 3) {
    nv1 = p.nv[1];
    d2 = 2 * nv1;
    g2.V = 1;
    for (int m = 0; m < 4; ++m) { g2.L[m] = g1.L[m] / p.agg[1][m]; g2.V *= g2.L[m]; }
    int nb[4];
    for (int m = 0; m < 4; ++m) nb[m] = g1.L[m] / p.sap_block1[m];
    build_colours(nb, blist1);
  }
}

template <typename T, typename S>
Hier<T, S>::~Hier() {
  drop_graphs();
  if (cap_st) (void)hipStreamDestroy(cap_st);
}

template <typename T, typename S>
void Hier<T, S>::drop_graphs() {
  for (GraphEntry& e : graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  graphs.clear();
}

// The intermediate-level solve of a fine cycle always reads rc1 and writes
// ec1, and its launch schedule depends only on the hierarchy and the
// right-hand-side count (fixed step counts, device-side convergence masks),
// so it is captured as a HIP graph and replayed.  A key is captured on its
// second use, so one-off calls never pay for the capture; the graphs hold
// the hierarchy's buffer addresses and are dropped whenever those may move.
// Returns false when the call must run eagerly.
template <typename T, typename S>
bool Hier<T, S>::coarse_solve_graph(int nrhs, const double* mu) {
  size_t k = 0;
  while (k < graphs.size() && !(graphs[k].nrhs == nrhs && graphs[k].mu == mu)) ++k;
  if (k == graphs.size()) graphs.push_back({nrhs, mu, 0, nullptr, 0, 0});
  if (!graphs[k].exec) {
    if (++graphs[k].calls < 2) return false;
    // capture runs no kernels: the host-side step counts it adds are the
    // counts of one replay
    const long l2_0 = stats_l2, cs_0 = stats_coarsest;
    if (!cap_st) HIPCHK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
    const hipStream_t saved = c->st;
    hipGraph_t gr = nullptr;
    c->st = cap_st;
    capturing = true;
    try {
      HIPCHK(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed));
      coarse_solve(1, rc1.p, ec1.p, nrhs, mu);
      HIPCHK(hipStreamEndCapture(cap_st, &gr));
    } catch (...) {
      hipGraph_t partial = nullptr;
      (void)hipStreamEndCapture(cap_st, &partial);
      if (partial) (void)hipGraphDestroy(partial);
      c->st = saved;
      capturing = false;
      throw;
    }
    c->st = saved;
    capturing = false;
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIPCHK(e);
    graphs[k].exec = ex;
    graphs[k].l2_steps = stats_l2 - l2_0;
    graphs[k].coarsest_steps = stats_coarsest - cs_0;
    stats_l2 = l2_0;
    stats_coarsest = cs_0;
  }
  HIPCHK(hipGraphLaunch(graphs[k].exec, c->st));
  stats_l2 += graphs[k].l2_steps;
  stats_coarsest += graphs[k].coarsest_steps;
  return true;
}

template <typename T, typename S>
void Hier<T, S>::build_colours(const int nb[4], DevArr<int> out[2]) {
  std::vector<int> lists[2];
  for (int b3 = 0; b3 < nb[3]; ++b3)
    for (int b2 = 0; b2 < nb[2]; ++b2)
      for (int b1 = 0; b1 < nb[1]; ++b1)
        for (int b0 = 0; b0 < nb[0]; ++b0) {
          int id = ((b3 * nb[2] + b2) * nb[1] + b1) * nb[0] + b0;
          lists[(b0 + b1 + b2 + b3) & 1].push_back(id);
        }
  for (int cidx = 0; cidx < 2; ++cidx) {
    out[cidx].alloc(std::max<size_t>(1, lists[cidx].size()));
    if (!lists[cidx].empty())
      HIPCHK(hipMemcpy(out[cidx].p, lists[cidx].data(), lists[cidx].size() * sizeof(int), hipMemcpyHostToDevice));
    out[cidx].count = (int)lists[cidx].size();
  }
}

template <typename T, typename S>
void Hier<T, S>::ensure(int nrhs) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  // the setup batches chunk(l) test vectors (all of them unless the
  // memory plan asks for fewer)
  int need = std::max(nrhs, nlev >= 2 ? chunk(0) : 0);
  if (nlev >= 3) need = std::max(need, chunk(1));
  if (need <= cap) return;
  drop_graphs();
  cap = need;
  red_partial.alloc(1024 * (size_t)cap);
  red_out.alloc(cap);
  red_inv.alloc(cap);
  if (nlev >= 2) {
    rc1.alloc((size_t)cap * g1.V * d1);
    ec1.alloc((size_t)cap * g1.V * d1);
    if (nlev == 2) K1.ensure(g1.V * d1, p.coarsest_iters, cap, false, st);
    else K1.ensure(g1.V * d1, p.l2_iters, cap, true, st);
  }
  if (nlev >= 3) {
    rc2.alloc((size_t)cap * g2.V * d2);
    ec2.alloc((size_t)cap * g2.V * d2);
    tmp1.alloc((size_t)cap * g1.V * d1);
    K2.ensure(g2.V * d2, p.coarsest_iters, cap, false, st);
    for (int k = 0; k < 2; ++k) {
      sap_rho[k].alloc((size_t)cap * g1.V * d1);
      sap_q[k].alloc((size_t)cap * g1.V * d1);
      sap_part[k].alloc(3 * (size_t)g1.V * cap);
    }
  }
  // coarsest level: persistent GMRES workspace
  {
    const CoarseGeom& gc = nlev >= 3 ? g2 : g1;
    const int dc = nlev >= 3 ? d2 : d1;
    if (nlev >= 2) {
      (void)dc;
      cg_dws.alloc(coarsest_ws_doubles(cap, p.coarsest_iters, coarsest_groups(gc.V)));
      cg_iws.alloc(coarsest_ws_ints(cap));
      HIPCHK(hipMemsetAsync(cg_iws.p, 0, cg_iws.bytes(), st));   // barrier counters start at zero
    }
  }
}

// Counters since the last call: host-side step counts of the generic
// Krylov cycles (and of graph replays) plus the persistent coarsest
// kernels' device counters (iterations summed over right-hand sides,
// launches, second Gram-Schmidt passes, barrier waits that gave up).
template <typename T, typename S>
HierBase::Counters Hier<T, S>::take_counters() {
  Counters k;
  k.l2 = stats_l2;
  k.coarsest = stats_coarsest;
  stats_l2 = stats_coarsest = 0;
  if (cg_iws.p) {
    int h[6] = {0, 0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, cg_iws.p + 2, sizeof(h), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (h[0] | h[1] | h[2] | h[5]) {
      HIPCHK(hipMemsetAsync(cg_iws.p + 2, 0, 3 * sizeof(int), c->st));
      HIPCHK(hipMemsetAsync(cg_iws.p + 7, 0, sizeof(int), c->st));
    }
    k.timeouts = h[0];
    k.coarsest += h[1];
    k.coarsest_calls = h[2];
    k.reorth = h[5];
  }
  return k;
}

template <typename T, typename S>
void Hier<T, S>::flag_barrier_timeout() {
  ensure(1);
  const int one = 1;
  HIPCHK(hipMemcpyAsync(cg_iws.p + 2, &one, sizeof(int), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

template <typename T, typename S>
void Hier<T, S>::dc_apply(int level, const cplx<T>* in, cplx<T>* out, int nrhs, const double* mu) {
  if (level == 1) launch_coarse_apply<T, S>(g1, d1, Dc1.p, in, out, nrhs, mu, c->st);
  else launch_coarse_apply<T, S>(g2, d2, Dc2.p, in, out, nrhs, mu, c->st);
}

template <typename T, typename S>
void Hier<T, S>::sap(int level, const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu, int sweeps) {
  const tmamg_params& p = c->par;
  for (int k = 0; k < sweeps; ++k)
    for (int col = 0; col < 2; ++col) {
      if (level == 0) {
        if (blist0[col].count == 0) continue;
        launch_sap_fine<T>(fop, eta, z, nrhs, mu, blist0[col].p, blist0[col].count, p.mr_steps, c->st,
                           nrhs == 2 ? nd_eps : 0.0);
      } else {
        if (blist1[col].count == 0) continue;
        launch_sap_coarse<T, S>(g1, d1, p.sap_block1, Dc1.p, eta, z, nrhs, mu, blist1[col].p, blist1[col].count,
                                p.mr_steps, c->st);
      }
    }
}

// Coarse-level SAP: site-per-workgroup launches with fused MR steps when
// the shape is covered, else one launch per colour and sweep.
template <typename T, typename S>
void Hier<T, S>::sap_level1(const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu, int sweeps) {
  const tmamg_params& p = c->par;
  cplx<T>* const rho[2] = {sap_rho[0].p, sap_rho[1].p};
  cplx<T>* const q[2] = {sap_q[0].p, sap_q[1].p};
  double* const part[2] = {sap_part[0].p, sap_part[1].p};
  if (use_coop && sweeps > 0 &&
      launch_sap_coarse_fused<T, S>(g1, d1, p.sap_block1, Dc1.p, eta, z, nrhs, mu, blist1[0].p, blist1[0].count,
                                    blist1[1].p, blist1[1].count, sweeps, p.mr_steps, rho, q, part,
                                    (long)sap_part[0].n, c->st))
    return;
  sap(1, eta, z, nrhs, mu, sweeps);
}

// Eq. (1): z = P D_c^-1 P^dag v (approximately), then k SAP sweeps on D z = v.
template <typename T, typename S>
void Hier<T, S>::precond(int level, const cplx<T>* v, cplx<T>* z, int nrhs, const double* mu) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  PhaseTimer& tmr = c->timer;
  if (level == 0) {
    if (nlev == 1) {
      launch_fill_zero(z, (size_t)nrhs * 12 * c->fg.V * sizeof(cplx<T>), st);
    } else {
      hipEvent_t e0 = tmr.begin(st);
      launch_restrict_fine<T, S>(c->fg, P0.p, nv0, v, rc1.p, nrhs, st);
      tmr.end(PhaseTimer::FINE_TRANSFER, e0, st);
      e0 = tmr.begin(st);
      coarse_solve(1, rc1.p, ec1.p, nrhs, mu);
      tmr.end(PhaseTimer::L1_SOLVE, e0, st);
      e0 = tmr.begin(st);
      launch_prolong_fine<T, S>(c->fg, P0.p, nv0, ec1.p, z, nrhs, st);
      tmr.end(PhaseTimer::FINE_TRANSFER, e0, st);
    }
    hipEvent_t e1 = tmr.begin(st);
    sap(0, v, z, nrhs, mu, p.sap_sweeps[0]);
    tmr.end(PhaseTimer::FINE_SAP, e1, st);
  } else {
    launch_restrict_coarse<T, S>(g1, d1, p.agg[1], P1.p, nv1, v, rc2.p, nrhs, st);
    hipEvent_t e0 = tmr.begin(st);
    coarse_solve(2, rc2.p, ec2.p, nrhs, mu);
    tmr.end(PhaseTimer::COARSEST, e0, st);
    launch_prolong_coarse<T, S>(g1, d1, p.agg[1], P1.p, nv1, ec2.p, z, nrhs, st);
    e0 = tmr.begin(st);
    sap_level1(v, z, nrhs, mu, p.sap_sweeps[1]);
    tmr.end(PhaseTimer::L1_SAP, e0, st);
  }
}

// Doublet (Sec. 1.1, Eq. (2)): with P_ND = P x I_2 and P^dag P = I the
// coarse operator is D_ND,c = P_ND^dag D_ND P_ND = [[D_c(mubar), -epsbar],
// [-epsbar, D_c(-mubar)]]: the two flavours' coarse fields (a pair of
// right-hand sides) are solved as one system whose operator is the
// flavour's own D_c plus -epsbar times the other flavour's field.
template <typename T, typename S>
void Hier<T, S>::coarse_solve_nd(int level, const cplx<T>* rhs, cplx<T>* sol, const double* mu) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  const long n = level == 1 ? g1.V * d1 : g2.V * d2;
  const double eps = nd_eps;
  const bool coarsest = level == nlev - 1;
  Krylov<T>& K = level == 1 ? KN1 : KN2;
  // the coupled coarsest GMRES takes twice the steps of one flavour's: each
  // step applies D_c to both flavours, so the operator work equals that of
  // the two flavours' separate solves
  const int csteps = std::min(2 * p.coarsest_iters, 127);
  K.ensure(2 * n, coarsest ? csteps : p.l2_iters, 1, !coarsest, st);
  launch_fill_zero(sol, (size_t)2 * n * sizeof(cplx<T>), st);
  OpFn<T> A = [this, level, mu, n, eps](const cplx<T>* in, cplx<T>* out) {
    dc_apply(level, in, out, 2, mu);
    launch_flavour_couple<T>(in, out, -eps, n, c->st);
  };
  if (coarsest) {
    stats_coarsest += krylov_cycle<T>(K, A, nullptr, rhs, sol, 1, csteps, p.coarsest_tol, nullptr, false, nullptr,
                                      st);
  } else {
    OpFn<T> M = [this, mu](const cplx<T>* in, cplx<T>* out) { precond(1, in, out, 2, mu); };
    stats_l2 += krylov_cycle<T>(K, A, &M, rhs, sol, 1, p.l2_iters, p.l2_tol, nullptr, false, nullptr, st);
  }
}

template <typename T, typename S>
void Hier<T, S>::coarse_solve(int level, const cplx<T>* rhs, cplx<T>* sol, int nrhs, const double* mu) {
  const tmamg_params& p = c->par;
  if (nd_eps != 0.0 && nrhs == 2) {
    coarse_solve_nd(level, rhs, sol, mu);
    return;
  }
  if (level == 1 && nlev >= 3 && p.use_graph && !capturing && !c->timer.on && rhs == rc1.p && sol == ec1.p &&
      coarse_solve_graph(nrhs, mu))
    return;
  hipStream_t st = c->st;
  long n = level == 1 ? g1.V * d1 : g2.V * d2;
  launch_fill_zero(sol, (size_t)nrhs * n * sizeof(cplx<T>), st);
  Krylov<T>& K = level == 1 ? K1 : K2;
  OpFn<T> A = [this, level, nrhs, mu](const cplx<T>* in, cplx<T>* out) { dc_apply(level, in, out, nrhs, mu); };
  if (level == nlev - 1) {
    const CoarseGeom& gc = level == 1 ? g1 : g2;
    const int dc = level == 1 ? d1 : d2;
    const SPair* Dc = level == 1 ? Dc1.p : Dc2.p;
    if (use_coop && launch_coarsest_gmres<T, S>(gc, dc, Dc, rhs, sol, nrhs, mu, p.coarsest_iters, p.coarsest_tol,
                                                K.V.p, K.w.p, cg_dws.p, cg_dws.n, cg_iws.p, cg_iws.n, st))
      return;
    int it = krylov_cycle<T>(K, A, nullptr, rhs, sol, nrhs, p.coarsest_iters, p.coarsest_tol, nullptr, false,
                             nullptr, st);
    stats_coarsest += it;
  } else {
    OpFn<T> M = [this, nrhs, mu](const cplx<T>* in, cplx<T>* out) { precond(1, in, out, nrhs, mu); };
    int it = krylov_cycle<T>(K, A, &M, rhs, sol, nrhs, p.l2_iters, p.l2_tol, nullptr, false, nullptr, st);
    stats_l2 += it;
  }
}

template <typename T, typename S>
void Hier<T, S>::normalize(cplx<T>* v, long n, int nrhs) {
  hipStream_t st = c->st;
  int NB = reduce_blocks(n);
  launch_norm2(v, n, nrhs, red_partial.p, NB, nullptr, st);
  launch_finalize_real(red_partial.p, nrhs, NB, red_out.p, st);
  hipLaunchKernelGGL(k_rsqrt, dim3((nrhs + 63) / 64), dim3(64), 0, st, red_out.p, red_inv.p, nrhs);
  launch_scale_dev(v, v, red_inv.p, n, nrhs, nullptr, st);
}

template <typename T, typename S>
void Hier<T, S>::build(int l) {
  hipStream_t st = c->st;
  const tmamg_params& p = c->par;
  drop_graphs();
  hipEvent_t e0 = c->timer.begin(st);
  build_inner(l);
  c->timer.end(PhaseTimer::SETUP_BUILD, e0, st);
}

template <typename T, typename S>
void Hier<T, S>::build_inner(int l) {
  hipStream_t st = c->st;
  const tmamg_params& p = c->par;
  if (l == 0) {
    launch_gs_fine<T, S>(c->fg, tv0.p, nv0, P64.p, P0.p, st);
    if (!gal_ws.p) {
      // up to 16 columns per pass within 4 GiB
      const size_t per_col = galerkin_ws_per_column(c->fg);
      const size_t cap_cols = std::max<size_t>(1, ((size_t)4 << 30) / (per_col * sizeof(cplx<T>)));
      gal_ws.alloc(per_col * std::min<size_t>({cap_cols, (size_t)16, (size_t)(2 * nv0)}));
    }
    launch_galerkin_fine<T, S>(fop, P0.p, nv0, Dc1.p, gal_ws.p, gal_ws.n, st);
  } else {
    launch_gs_coarse<T, S>(g1, d1, p.agg[1], tv1.p, nv1, P64.p, P1.p, st);
    launch_galerkin_coarse<T, S>(g1, d1, p.agg[1], Dc1.p, P1.p, nv1, Dc2.p, st);
  }
}

template <typename T, typename S>
void Hier<T, S>::galerkin_only(int l) {
  const tmamg_params& p = c->par;
  if (l == 1) launch_galerkin_coarse<T, S>(g1, d1, p.agg[1], Dc1.p, P1.p, nv1, Dc2.p, c->st);
}

template <typename T, typename S>
void Hier<T, S>::setup(double mu) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  if (nlev < 2) return;
  const long n0 = 12 * c->fg.V;
  tv0.alloc((size_t)nv0 * n0);
  P0.alloc((size_t)nv0 * n0);
  Dc1.alloc((size_t)g1.V * 9 * d1 * d1);
  size_t p64 = 0;
  if (nlev >= 3) {
    tv1.alloc((size_t)nv1 * g1.V * d1);
    P1.alloc((size_t)nv1 * g1.V * d1);
    Dc2.alloc((size_t)g2.V * 9 * d2 * d2);
  }
  (void)p64;
  ensure(std::max(chunk(0), nlev >= 3 ? chunk(1) : 0));
  setup_workspace();
  mu_setup.alloc(std::max(nv0, nv1));
  int nmax = std::max(nv0, nv1);
  hipLaunchKernelGGL(k_fill_double, dim3(1), dim3(64), 0, st, mu_setup.p, mu, nmax);
  // level-0 start vectors
  if (c->inject0.p) launch_convert<double, T>(c->inject0.p, tv0.p, (long)nv0 * n0, st);
  else launch_random<T>(tv0.p, (long)nv0 * n0, p.seed, st);
  smooth_vectors(0);
  build(0);
  if (nlev >= 3) {
    long n1 = g1.V * d1;
    if (c->inject1.p) launch_convert<double, T>(c->inject1.p, tv1.p, (long)nv1 * n1, st);
    else launch_random<T>(tv1.p, (long)nv1 * n1, p.seed + 7919, st);
    smooth_vectors(1);
    build(1);
  }
  for (int it = 0; it < p.setup_iters; ++it) setup_iteration();
  release_setup_workspace();
}

// Test vectors treated at once on level l (the memory plan's setup_chunk).
template <typename T, typename S>
int Hier<T, S>::chunk(int l) const {
  const int nv = l == 0 ? nv0 : nv1;
  const int ch = c->par.setup_chunk;
  return ch > 0 && ch < nv ? ch : nv;
}

// The setup's work buffers: the fine level's batch of smoothed or cycled
// test vectors and the FP64 scratch of the orthonormalisation (the fine
// level's Cholesky QR needs none for the vector counts used here).
template <typename T, typename S>
void Hier<T, S>::setup_workspace() {
  const long n0 = 12 * c->fg.V;
  size_t p64 = gs_fine_needs_fp64_copy(nv0) ? (size_t)nv0 * n0 : 0;
  if (nlev >= 3) p64 = std::max(p64, (size_t)nv1 * g1.V * d1);
  if (!P64.p) P64.alloc(std::max<size_t>(p64, 1));
  if (!tvtmp.p) tvtmp.alloc((size_t)chunk(0) * n0);
}

template <typename T, typename S>
void Hier<T, S>::release_setup_workspace() {
  HIPCHK(hipStreamSynchronize(c->st));
  tvtmp.release();
  P64.release();
  gal_ws.release();
  if (!c->par.keep_test_vectors) tv0.release();
}

// Initial phase: v <- SAP(v) from zero, normalised, init_smooth times
// (test vectors in batches of chunk(l), each treated alone).
template <typename T, typename S>
void Hier<T, S>::smooth_vectors(int l) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  const long n = l == 0 ? 12 * c->fg.V : g1.V * d1;
  const int nv = l == 0 ? nv0 : nv1, ch = chunk(l);
  cplx<T>* v = l == 0 ? tv0.p : tv1.p;
  cplx<T>* w = l == 0 ? tvtmp.p : tmp1.p;
  for (int k = 0; k < p.init_smooth; ++k) {
    for (int i0 = 0; i0 < nv; i0 += ch) {
      const int nc = std::min(ch, nv - i0);
      cplx<T>* vc = v + (size_t)i0 * n;
      launch_fill_zero(w, (size_t)nc * n * sizeof(cplx<T>), st);
      if (l == 0) sap(0, vc, w, nc, mu_setup.p, p.sap_sweeps[0]);
      else sap_level1(vc, w, nc, mu_setup.p, p.sap_sweeps[1]);
      HIPCHK(hipMemcpyAsync(vc, w, (size_t)nc * n * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
      normalize(vc, n, nc);
    }
  }
}

// v_i <- B_MG v_i on each level in turn (normalised), rebuilding P and D_c;
// the Galerkin operator below a rebuilt one is recomputed at once from its
// current P so the next level's update uses a consistent cycle.
template <typename T, typename S>
void Hier<T, S>::setup_iteration() {
  hipStream_t st = c->st;
  setup_workspace();
  for (int l = 0; l < nlev - 1; ++l) {
    const long n = l == 0 ? 12 * c->fg.V : g1.V * d1;
    const int nv = l == 0 ? nv0 : nv1, ch = chunk(l);
    cplx<T>* v = l == 0 ? tv0.p : tv1.p;
    cplx<T>* w = l == 0 ? tvtmp.p : tmp1.p;
    for (int i0 = 0; i0 < nv; i0 += ch) {
      const int nc = std::min(ch, nv - i0);
      cplx<T>* vc = v + (size_t)i0 * n;
      precond(l, vc, w, nc, mu_setup.p);
      HIPCHK(hipMemcpyAsync(vc, w, (size_t)nc * n * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
      normalize(vc, n, nc);
    }
    build(l);
    if (l + 2 < nlev) galerkin_only(l + 1);
  }
}

template struct Hier<double, double>;
template struct Hier<float, float>;
template struct Hier<float, __hip_bfloat16>;
template struct Hier<float, __half>;
template int krylov_cycle<double>(Krylov<double>&, const OpFn<double>&, const OpFn<double>*, const cplx<double>*,
                                  cplx<double>*, int, int, double, const double*, bool, int*, hipStream_t);
template int krylov_cycle<float>(Krylov<float>&, const OpFn<float>&, const OpFn<float>*, const cplx<float>*,
                                 cplx<float>*, int, int, double, const double*, bool, int*, hipStream_t);
template struct Krylov<double>;
template struct Krylov<float>;
