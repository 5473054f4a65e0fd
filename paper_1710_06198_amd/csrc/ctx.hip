// Context, outer solvers and the C ABI entry points.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>
#include <cstdlib>
#include <mutex>

using clk = std::chrono::steady_clock;

__global__ void k_fill_double(double* p, double v, int n);

// ------------------------------------------------------------------ Hier: typed hooks
template <typename T, typename S>
void Hier<T, S>::precond_d(const cplx<double>* v, cplx<double>* z, int nrhs, const double* mu) {
  if constexpr (std::is_same<T, double>::value) precond(0, v, z, nrhs, mu);
  else throw TmError{TMAMG_ESTATE, "FP64 cycle requested from an FP32 hierarchy"};
}
template <typename T, typename S>
void Hier<T, S>::precond_f(const cplx<float>* v, cplx<float>* z, int nrhs, const double* mu) {
  if constexpr (std::is_same<T, float>::value) precond(0, v, z, nrhs, mu);
  else throw TmError{TMAMG_ESTATE, "FP32 cycle requested from an FP64 hierarchy"};
}

template <typename T, typename S>
void Hier<T, S>::rebuild() {
  if (nlev < 2) return;
  setup_workspace();
  build(0);
  if (nlev >= 3) build(1);
}

template <typename T, typename S>
void Hier<T, S>::test_op(int op, int level, const void* in_, void* out_, int nrhs, const double* mu) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  ensure(nrhs);
  const cplx<T>* in = static_cast<const cplx<T>*>(in_);
  cplx<T>* out = static_cast<cplx<T>*>(out_);
  auto need = [&](bool ok) { if (!ok) throw TmError{TMAMG_EINVAL, "operator not available on this level"}; };
  switch (op) {
    case TMAMG_OP_PROLONG:
      need(level >= 1 && level < nlev);
      if (level == 1) launch_prolong_fine<T, S>(c->fg, P0.p, nv0, in, out, nrhs, st);
      else launch_prolong_coarse<T, S>(g1, d1, p.agg[1], P1.p, nv1, in, out, nrhs, st);
      break;
    case TMAMG_OP_RESTRICT:
      need(level >= 0 && level < nlev - 1);
      if (level == 0) launch_restrict_fine<T, S>(c->fg, P0.p, nv0, in, out, nrhs, st);
      else launch_restrict_coarse<T, S>(g1, d1, p.agg[1], P1.p, nv1, in, out, nrhs, st);
      break;
    case TMAMG_OP_DC:
      need(level >= 1 && level < nlev);
      dc_apply(level, in, out, nrhs, mu);
      break;
    case TMAMG_OP_SAP: {
      need(level == 0 || (level == 1 && nlev >= 3));
      long n = level == 0 ? 12 * c->fg.V : g1.V * d1;
      launch_fill_zero(out, (size_t)nrhs * n * sizeof(cplx<T>), st);
      if (level == 0) sap(0, in, out, nrhs, mu, p.sap_sweeps[0]);
      else sap_level1(in, out, nrhs, mu, p.sap_sweeps[1]);
      break;
    }
    case TMAMG_OP_PREC:
      need(level == 0 || (level == 1 && nlev >= 3));
      precond(level, in, out, nrhs, mu);
      break;
    case TMAMG_OP_COARSEST:
      need(level >= 1 && level == nlev - 1);
      coarse_solve(level, in, out, nrhs, mu);
      break;
    case TMAMG_OP_SAPND: {
      need(level == 0 && nrhs == 2);
      launch_fill_zero(out, (size_t)2 * 12 * c->fg.V * sizeof(cplx<T>), st);
      sap(0, in, out, 2, mu, p.sap_sweeps[0]);
      break;
    }
    case TMAMG_OP_DCND: {
      need(level >= 1 && level < nlev && nrhs == 2);
      const long n = level == 1 ? g1.V * d1 : g2.V * d2;
      dc_apply(level, in, out, 2, mu);
      launch_flavour_couple<T>(in, out, -nd_eps, n, st);
      break;
    }
    default:
      throw TmError{TMAMG_EINVAL, "unknown operator"};
  }
}

template <typename T, typename S>
void Hier<T, S>::export_P(int level, cplx<double>* out) {
  hipStream_t st = c->st;
  if (level == 0) {
    if (nlev < 2) throw TmError{TMAMG_EINVAL, "no coarsening"};
    long n0 = 12 * c->fg.V;
    DevArr<cplx<double>> tmp;
    tmp.alloc((size_t)nv0 * n0);
    launch_store_to64<S>(P0.p, tmp.p, (long)nv0 * n0, st);
    launch_spinor_to_canonical<double>(c->fg, tmp.p, out, nv0, st);
    HIPCHK(hipStreamSynchronize(st));
  } else {
    if (nlev < 3) throw TmError{TMAMG_EINVAL, "no second coarsening"};
    launch_store_to64<S>(P1.p, out, (long)nv1 * g1.V * d1, st);
  }
}
template <typename T, typename S>
void Hier<T, S>::export_Dc(int level, cplx<double>* out) {
  if (level == 1 && nlev >= 2) launch_store_to64<S>(Dc1.p, out, (long)g1.V * 9 * d1 * d1, c->st);
  else if (level == 2 && nlev >= 3) launch_store_to64<S>(Dc2.p, out, (long)g2.V * 9 * d2 * d2, c->st);
  else throw TmError{TMAMG_EINVAL, "no such coarse level"};
}

template <typename T, typename S>
double Hier<T, S>::time_kernel(int kernel, int nrhs, int reps) {
  const tmamg_params& p = c->par;
  hipStream_t st = c->st;
  ensure(nrhs);
  const long n0 = 12 * c->fg.V;
  auto need = [&](bool ok) { if (!ok) throw TmError{TMAMG_EINVAL, "kernel not available in this hierarchy"}; };
  DevArr<cplx<T>> a, b;
  DevArr<double> mu;
  mu.alloc(nrhs);
  hipLaunchKernelGGL(k_fill_double, dim3((nrhs + 63) / 64), dim3(64), 0, st, mu.p, c->mu, nrhs);
  switch (kernel) {
    case TMAMG_K_SAP0: {
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * n0);
      launch_random<T>(a.p, (long)nrhs * n0, 11, st);
      launch_fill_zero(b.p, b.bytes(), st);
      return time_launches(st, reps, [&]() {
        launch_sap_fine<T>(fop, a.p, b.p, nrhs, mu.p, blist0[0].p, blist0[0].count, p.mr_steps, st);
      });
    }
    case TMAMG_K_RESTRICT0:
    case TMAMG_K_PROLONG0: {
      need(nlev >= 2);
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * g1.V * d1);
      launch_random<T>(a.p, (long)nrhs * n0, 12, st);
      launch_random<T>(b.p, (long)nrhs * g1.V * d1, 13, st);
      if (kernel == TMAMG_K_RESTRICT0)
        return time_launches(st, reps, [&]() { launch_restrict_fine<T, S>(c->fg, P0.p, nv0, a.p, b.p, nrhs, st); });
      return time_launches(st, reps, [&]() { launch_prolong_fine<T, S>(c->fg, P0.p, nv0, b.p, a.p, nrhs, st); });
    }
    case TMAMG_K_DC1:
    case TMAMG_K_DC2: {
      int lv = kernel == TMAMG_K_DC1 ? 1 : 2;
      need(nlev > lv);
      long n = lv == 1 ? g1.V * d1 : g2.V * d2;
      a.alloc((size_t)nrhs * n);
      b.alloc((size_t)nrhs * n);
      launch_random<T>(a.p, (long)nrhs * n, 14, st);
      return time_launches(st, reps, [&]() { dc_apply(lv, a.p, b.p, nrhs, mu.p); });
    }
    case TMAMG_K_SAP1: {
      need(nlev >= 3);
      long n = g1.V * d1;
      a.alloc((size_t)nrhs * n);
      b.alloc((size_t)nrhs * n);
      launch_random<T>(a.p, (long)nrhs * n, 15, st);
      launch_fill_zero(b.p, b.bytes(), st);
      return time_launches(st, reps, [&]() { sap_level1(a.p, b.p, nrhs, mu.p, 1); });
    }
    default:
      throw TmError{TMAMG_EINVAL, "unknown kernel id"};
  }
}

template struct Hier<double, double>;
template struct Hier<float, float>;
template struct Hier<float, __hip_bfloat16>;
template struct Hier<float, __half>;

// ------------------------------------------------------------------ context
static void check(bool ok, const std::string& msg) {
  if (!ok) throw TmError{TMAMG_EINVAL, msg};
}

static bool even_or_one(int n) { return n == 1 || n % 2 == 0; }

Ctx::Ctx(const tmamg_lattice& l, const tmamg_params& p, hipStream_t s, const tmamg_allocator* a)
    : lat(l), par(p), st(s) {
  if (a) {
    check(a->alloc != nullptr && a->free != nullptr, "an allocator needs both alloc and free");
    dalloc.alloc = a->alloc;
    dalloc.free = a->free;
    dalloc.user = a->user;
    dalloc.st = s;
  }
  check(p.nlevels >= 0 && p.nlevels <= 3, "nlevels must be 0..3");
  check(p.restart >= 1 && p.restart <= 127, "restart must be 1..127");
  check(p.max_iter >= 1, "max_iter must be positive");
  check(p.mr_steps >= 0 && p.sap_sweeps[0] >= 0 && p.sap_sweeps[1] >= 0, "negative smoother counts");
  check(p.precision == TMAMG_FP64 || p.precision == TMAMG_MIXED, "precision");
  check(p.use_graph == 0 || p.use_graph == 1, "use_graph must be 0 or 1");
  check(p.nd_coarse_coupling == 0 || p.nd_coarse_coupling == 1, "nd_coarse_coupling must be 0 or 1");
  check(p.setup_chunk >= 0, "setup_chunk must be >= 0");
  check(p.keep_test_vectors == 0 || p.keep_test_vectors == 1, "keep_test_vectors must be 0 or 1");
  if (p.precision == TMAMG_MIXED)
    check(p.storage == TMAMG_STORE_FP32 || p.storage == TMAMG_STORE_BF16 || p.storage == TMAMG_STORE_FP16,
          "mixed precision stores P and D_c in fp32, bf16 or fp16");
  int bvol = 1;
  for (int m = 0; m < 4; ++m) {
    check(l.dims[m] >= 1 && p.agg[0][m] >= 1, "dims and aggregates must be positive");
    check(l.dims[m] % p.agg[0][m] == 0, "lattice extents must be multiples of the first aggregate");
    bvol *= p.agg[0][m];
  }
  check(bvol % 64 == 0 && bvol <= 256, "the fine aggregate/SAP block must hold 64, 128, 192 or 256 sites");
  fg.V = 1;
  for (int m = 0; m < 4; ++m) {
    fg.L[m] = l.dims[m];
    fg.B[m] = p.agg[0][m];
    fg.NB[m] = l.dims[m] / p.agg[0][m];
    fg.V *= l.dims[m];
    check(even_or_one(fg.NB[m]), "SAP needs an even number of fine blocks (or one) per dimension");
  }
  fg.bvol = bvol;
  fg.nblocks = (int)(fg.V / bvol);
  fg.lstride[0] = 1;
  fg.bstride[0] = 1;
  for (int m = 1; m < 4; ++m) {
    fg.lstride[m] = fg.lstride[m - 1] * fg.B[m - 1];
    fg.bstride[m] = fg.bstride[m - 1] * fg.NB[m - 1];
  }
  if (p.nlevels >= 2) {
    check(p.nv[0] >= 1 && p.nv[0] <= 64, "nv[0] must be 1..64");
    check(p.coarsest_iters >= 1 && p.coarsest_iters <= 127, "coarsest_iters must be 1..127");
  }
  if (p.nlevels >= 3) {
    check(p.nv[1] >= 1 && p.nv[1] <= 64, "nv[1] must be 1..64");
    check(p.l2_iters >= 1 && p.l2_iters <= 127, "l2_iters must be 1..127");
    int na = 1, nbs = 1;
    for (int m = 0; m < 4; ++m) {
      int L1 = fg.NB[m];
      check(p.agg[1][m] >= 1 && L1 % p.agg[1][m] == 0, "coarse extents must be multiples of the second aggregate");
      check(p.sap_block1[m] >= 1 && L1 % p.sap_block1[m] == 0, "coarse SAP block must tile the coarse lattice");
      check(even_or_one(L1 / p.sap_block1[m]), "coarse SAP needs an even number of blocks (or one) per dimension");
      na *= p.agg[1][m];
      nbs *= p.sap_block1[m];
    }
    // LDS budgets of the coarse Gram-Schmidt / Galerkin and coarse SAP kernels (64 KB per workgroup)
    check(na * p.nv[0] <= 768, "second aggregate too large (sites * nv[0] <= 768)");
    check(nbs * 2 * p.nv[0] <= 4000, "coarse SAP block too large (sites * dof <= 4000)");
  }
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&host_flags), 1024 * sizeof(int), hipHostMallocDefault));
  const char* tv = getenv("TMAMG_TIMING");
  timer.on = tv && tv[0] == '1';
}

Ctx::~Ctx() {
  if (host_flags) (void)hipHostFree(host_flags);
}

__global__ void k_unitarity(const cplx<double>* U, long V, double* out) {
  __shared__ double red[4];
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int mu = blockIdx.y;
  double dev = 0;
  if (s < V) {
    cplx<double> u[3][3];
    const cplx<double>* p = U + (size_t)mu * 9 * V + tsite((unsigned)s, 9);
    for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = p[k * FT];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cplx<double> a = mk(0.0, 0.0);
        for (int k = 0; k < 3; ++k) cfma(a, u[i][k], conj(u[j][k]));
        if (i == j) a.re -= 1.0;
        dev = fmax(dev, sqrt(norm2(a)));
      }
    if (!(dev == dev)) dev = 1e300;
  }
  for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.y * gridDim.x + blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Chiral blocks of sigma_{mu nu} = (i/2)[g_mu, g_nu] for the planes mu < nu
// (order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)); g_k = [[0, -i s_k], [i s_k, 0]],
// g_4 = [[0, 1], [1, 0]].  sigma commutes with g5, so only the two 2x2
// diagonal blocks (spins 0,1 and 2,3) are non-zero.
void sigma_blocks(double re[6][2][2][2], double im[6][2][2][2]) {
  using Cx = std::complex<double>;
  Cx g[4][4][4] = {};
  const Cx I(0, 1);
  Cx sig[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        g[k][a][2 + b] = -I * sig[k][a][b];
        g[k][2 + a][b] = I * sig[k][a][b];
      }
  for (int a = 0; a < 2; ++a) { g[3][a][2 + a] = 1; g[3][2 + a][a] = 1; }
  int pl = 0;
  for (int m = 0; m < 4; ++m)
    for (int n = m + 1; n < 4; ++n, ++pl) {
      Cx s4[4][4];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          Cx acc = 0;
          for (int k = 0; k < 4; ++k) acc += g[m][i][k] * g[n][k][j] - g[n][i][k] * g[m][k][j];
          s4[i][j] = 0.5 * I * acc;
        }
      for (int ch = 0; ch < 2; ++ch)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            re[pl][ch][a][b] = s4[2 * ch + a][2 * ch + b].real();
            im[pl][ch][a][b] = s4[2 * ch + a][2 * ch + b].imag();
          }
    }
}

void Ctx::load_links(const cplx<double>* U) {
  check(U != nullptr, "null link pointer");
  links64.alloc((size_t)4 * 9 * fg.V);
  bool mixed = par.precision == TMAMG_MIXED;
  if (mixed) links32.alloc((size_t)4 * 9 * fg.V);
  launch_convert_links(fg, U, links64.p, mixed ? links32.p : nullptr, lat.t_antiperiodic, st);
  // unitarity check
  unsigned nb = (unsigned)((fg.V + 255) / 256);
  DevArr<double> dv;
  dv.alloc((size_t)nb * 4);
  hipLaunchKernelGGL(k_unitarity, dim3(nb, 4), dim3(256), 0, st, links64.p, fg.V, dv.p);
  std::vector<double> h(nb * 4);
  HIPCHK(hipMemcpyAsync(h.data(), dv.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double mx = 0;
  for (double v : h) mx = std::max(mx, v);
  if (!(mx <= 1e-6)) throw TmError{TMAMG_ENUMERIC, "links are not unitary (max |U U^dag - 1| = " + std::to_string(mx) + ")"};
  // clover: A_s = (m0+4) + sum_{mu<nu} [c_sw (i/2) sigma_{mu nu}]_s Fhat_{mu nu}
  CloverCoef cc{};
  cc.diag = m0 + 4.0;
  double sre[6][2][2][2], sim[6][2][2][2];
  sigma_blocks(sre, sim);
  for (int pl = 0; pl < 6; ++pl)
    for (int ch = 0; ch < 2; ++ch)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          // c_sw (i/2) (re + i im)
          cc.re[pl][ch][a][b] = -0.5 * csw * sim[pl][ch][a][b];
          cc.im[pl][ch][a][b] = 0.5 * csw * sre[pl][ch][a][b];
        }
  clov64.alloc((size_t)72 * fg.V);
  if (mixed) clov32.alloc((size_t)72 * fg.V);
  launch_clover_build(fg, links64.p, cc, clov64.p, mixed ? clov32.p : nullptr, st);
  have_links = true;
}

// Counters of work outside a solve (setup, operator hooks): dropped, but a
// timed-out barrier wait still fails the call and retires the persistent
// coarse kernels.
HierBase::Counters Ctx::drain_counters() {
  const HierBase::Counters k = hier->take_counters();
  if (k.timeouts > 0) {
    hier->disable_persistent();
    throw TmError{TMAMG_EHIP, "a persistent coarse kernel's barrier wait timed out; the coarsest level uses the "
                              "generic kernels from now on"};
  }
  return k;
}

void Ctx::setup(const cplx<double>* U, double kappa_, double csw_, double mu_) {
  check(kappa_ > 0 && std::isfinite(kappa_), "kappa must be positive");
  check(std::isfinite(csw_) && std::isfinite(mu_), "csw and mu must be finite");
  auto t0 = clk::now();
  kappa = kappa_;
  csw = csw_;
  mu = mu_;
  m0 = 1.0 / (2.0 * kappa) - 4.0;
  load_links(U);
  if (par.precision == TMAMG_FP64) hier.reset(new Hier<double, double>(this));
  else if (par.storage == TMAMG_STORE_FP32) hier.reset(new Hier<float, float>(this));
  else if (par.storage == TMAMG_STORE_BF16) hier.reset(new Hier<float, __hip_bfloat16>(this));
  else hier.reset(new Hier<float, __half>(this));
  hier->setup(mu);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  {
    // the setup's own coarse iterations are not a solve's
    const HierBase::Counters k = drain_counters();
    if (timer.on)
      timer.report("setup", st, " level1_iters=" + std::to_string(k.l2) + " coarsest_iters=" +
                                  std::to_string(k.coarsest) + " coarsest_calls=" + std::to_string(k.coarsest_calls));
  }
  have_setup = true;
  t_setup = std::chrono::duration<double>(clk::now() - t0).count();
}

void Ctx::setup_update(const cplx<double>* U, int iters) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "setup_update before setup"};
  if (!hier->has_test_vectors())
    throw TmError{TMAMG_ESTATE, "the setup released its test vectors (keep_test_vectors = 0)"};
  check(iters >= 0, "iters must be >= 0");
  auto t0 = clk::now();
  load_links(U);
  hier->rebuild();
  for (int i = 0; i < iters; ++i) hier->setup_iteration();
  hier->release_setup_workspace();
  HIPCHK(hipStreamSynchronize(st));
  (void)drain_counters();
  t_setup = std::chrono::duration<double>(clk::now() - t0).count();
}

void Ctx::ensure(int nrhs) {
  if (nrhs <= cap) return;
  cap = nrhs;
  const long n = 12 * fg.V;
  b64.alloc((size_t)cap * n);
  x64.alloc((size_t)cap * n);
  r64.alloc((size_t)cap * n);
  t64.alloc((size_t)cap * n);
  mu_dev.alloc(cap);
  mu_cdev.alloc(cap);
  abstol_dev.alloc(cap);
  red_partial.alloc(1024 * (size_t)cap);
  red_out.alloc(2 * (size_t)cap);   // room for one complex result per right-hand side
  bool flex = par.nlevels >= 1;
  if (par.precision == TMAMG_FP64) {
    K64.ensure(n, par.restart, cap, flex, st);
  } else {
    r32.alloc((size_t)cap * n);
    e32.alloc((size_t)cap * n);
    K32.ensure(n, par.restart, cap, flex, st);
  }
  if (hier) hier->ensure(cap);
}

std::vector<double> Ctx::norms(const cplx<double>* v, int nrhs) {
  const long n = 12 * fg.V;
  int NB = reduce_blocks(n);
  launch_norm2(v, n, nrhs, red_partial.p, NB, nullptr, st);
  launch_finalize_real(red_partial.p, nrhs, NB, red_out.p, st);
  std::vector<double> h(nrhs);
  HIPCHK(hipMemcpyAsync(h.data(), red_out.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (double& x : h) x = std::sqrt(x);
  return h;
}

void Ctx::upload_mu(int nrhs, const double* mu_host) {
  std::vector<double> m(nrhs, mu);
  if (mu_host)
    for (int r = 0; r < nrhs; ++r) {
      check(std::isfinite(mu_host[r]), "non-finite twisted mass");
      m[r] = mu_host[r];
    }
  launch_set_doubles(mu_dev.p, m.data(), nrhs, st);
  mu_now = m;
}

// b64 holds the right-hand sides (internal layout); x64 receives the solutions.
// Outer loop: FP64 true residual r = b - D x at every restart (reliable update).
// FP64 mode: FGMRES(m) cycles on r with the FP64 cycle.  Mixed mode: the
// cycle's Krylov space, operator and multigrid run in FP32 (P, D_c in the
// storage type) on r rounded to FP32, stopped at inner_tol * ||r|| (defect
// correction); the correction is added to x in FP64.
// eps_nd set: the two right-hand sides are the flavours of one doublet
// system D_ND x = b (Sec. 1.1, Eq. 2), twisted masses +-mubar in mu_host and
// coupling -epsbar; one Krylov space spans both flavours, and the
// preconditioner is the multigrid cycle of each flavour's own D(+-mubar)
// (the coupling is left to the flexible outer iteration).
tmamg_status Ctx::solve_core(int nrhs, const double* mu_host, double tol, tmamg_info* info, const double* eps_nd,
                             bool guess) {
  const long n = 12 * fg.V;
  const bool nd = eps_nd != nullptr;
  const double eps = nd ? *eps_nd : 0.0;
  if (nd) check(nrhs == 2, "a doublet has two flavours");
  const int nk = nd ? 1 : nrhs;   // Krylov systems
  auto sys_norms = [&](const cplx<double>* v) {
    std::vector<double> h = norms(v, nrhs);
    if (nd) h = {std::hypot(h[0], h[1])};
    return h;
  };
  upload_mu(nrhs, mu_host);
  std::vector<double> bn = sys_norms(b64.p);
  for (double v : bn)
    if (!std::isfinite(v)) throw TmError{TMAMG_ENUMERIC, "right-hand side holds NaN/Inf"};
  const bool mixed = par.precision == TMAMG_MIXED;
  FineOp<double> o64 = op64();
  FineOp<float> o32 = mixed ? op32() : FineOp<float>{};
  const double* mu_d = mu_dev.p;
  if (guess && !nd) {
    // x64 holds the initial guess: r = b - D x0; a right-hand side whose
    // guess is worse than zero starts from zero
    launch_dslash<double>(o64, x64.p, t64.p, nrhs, mu_d, st);
    launch_xmy<double>(b64.p, t64.p, (long)nrhs * n, st);
    std::vector<double> rn0 = norms(t64.p, nrhs);
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(rn0[r])) throw TmError{TMAMG_ENUMERIC, "initial guess holds NaN/Inf"};
      if (rn0[r] > bn[r]) {
        launch_fill_zero(x64.p + (size_t)r * n, n * sizeof(cplx<double>), st);
        HIPCHK(hipMemcpyAsync(t64.p + (size_t)r * n, b64.p + (size_t)r * n, n * sizeof(cplx<double>),
                              hipMemcpyDeviceToDevice, st));
      }
    }
    std::swap(r64.p, t64.p);
  } else {
    launch_fill_zero(x64.p, (size_t)nrhs * n * sizeof(cplx<double>), st);
    HIPCHK(hipMemcpyAsync(r64.p, b64.p, (size_t)nrhs * n * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  }
  // the right-hand sides of the current cycle (all of them, or the ones
  // still above tol gathered into the first slots) and their twisted masses
  int cur_n = nrhs;
  const double* cur_mu = mu_d;
  OpFn<double> A64 = [&](const cplx<double>* in, cplx<double>* out) {
    hipEvent_t e0 = timer.begin(st);
    launch_dslash<double>(o64, in, out, cur_n, cur_mu, st);
    if (nd) launch_flavour_couple<double>(in, out, -eps, n, st);
    timer.end(PhaseTimer::OUTER_OP, e0, st);
  };
  OpFn<float> A32 = [&](const cplx<float>* in, cplx<float>* out) {
    hipEvent_t e0 = timer.begin(st);
    launch_dslash<float>(o32, in, out, cur_n, cur_mu, st);
    if (nd) launch_flavour_couple<float>(in, out, -eps, n, st);
    timer.end(PhaseTimer::OUTER_OP, e0, st);
  };
  OpFn<double> M64 = [&](const cplx<double>* in, cplx<double>* out) { hier->precond_d(in, out, cur_n, cur_mu); };
  OpFn<float> M32 = [&](const cplx<float>* in, cplx<float>* out) { hier->precond_f(in, out, cur_n, cur_mu); };
  Krylov<double>& k64 = nd ? KN64 : K64;
  Krylov<float>& k32 = nd ? KN32 : K32;
  // the coarse levels of a doublet's cycle carry the flavour coupling
  struct NdScope {
    HierBase* h;
    NdScope(HierBase* h_, double e) : h(h_) { h->nd_eps = e; }
    ~NdScope() { h->nd_eps = 0.0; }
  } nd_scope(hier.get(), (nd && par.nd_coarse_coupling) ? eps : 0.0);
  const bool use_m = par.nlevels >= 1;
  int iters = 0, cycles = 0;
  tmamg_status status = TMAMG_NOT_CONVERGED;
  double worst = 0;
  std::vector<double> at(nk);
  while (true) {
    std::vector<double> rn = sys_norms(r64.p);
    worst = 0;
    bool all = true;
    for (int r = 0; r < nk; ++r) {
      if (!std::isfinite(rn[r])) throw TmError{TMAMG_ENUMERIC, "residual became NaN/Inf"};
      double rel = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
      worst = std::max(worst, rel);
      all &= rel <= tol;
    }
    if (all) { status = TMAMG_OK; break; }
    if (iters >= par.max_iter) break;
    // this cycle's absolute targets
    for (int r = 0; r < nk; ++r)
      at[r] = mixed ? std::max(par.inner_tol * rn[r], 0.5 * tol * bn[r]) : 0.9 * tol * bn[r];
    // a right-hand side already at its target would sit idle in the cycle
    // (the Krylov steps skip it) while the operator and the multigrid cycle
    // still work on it: it stays out, the others are gathered into the first
    // slots, and their corrections are scattered back
    std::vector<int> act;
    if (!nd)
      for (int r = 0; r < nk; ++r)
        if (rn[r] > at[r]) act.push_back(r);
    const bool compact = !nd && !act.empty() && (int)act.size() < nk;
    const int na = compact ? (int)act.size() : nk;
    cur_n = compact ? na : nrhs;
    cur_mu = mu_d;
    if (compact) {
      std::vector<double> mc(na);
      for (int i = 0; i < na; ++i) mc[i] = mu_now[act[i]];
      launch_set_doubles(mu_cdev.p, mc.data(), na, st);
      cur_mu = mu_cdev.p;
    }
    auto set_abstol = [&]() {
      std::vector<double> ac(na);
      for (int i = 0; i < na; ++i) ac[i] = at[compact ? act[i] : i];
      launch_set_doubles(abstol_dev.p, ac.data(), na, st);
    };
    int it;
    if (!mixed) {
      set_abstol();
      if (compact) {
        c64.alloc(std::max(c64.n, (size_t)na * n));
        for (int i = 0; i < na; ++i)
          HIPCHK(hipMemcpyAsync(t64.p + (size_t)i * n, r64.p + (size_t)act[i] * n, n * sizeof(cplx<double>),
                                hipMemcpyDeviceToDevice, st));
        launch_fill_zero(c64.p, (size_t)na * n * sizeof(cplx<double>), st);
        it = krylov_cycle<double>(k64, A64, use_m ? &M64 : nullptr, t64.p, c64.p, na,
                                  std::min(par.restart, par.max_iter - iters), 0.0, abstol_dev.p, true, host_flags,
                                  st);
        for (int i = 0; i < na; ++i)
          launch_axpby<double>(c64.p + (size_t)i * n, x64.p + (size_t)act[i] * n, 1.0, 1.0, n, st);
      } else {
        it = krylov_cycle<double>(k64, A64, use_m ? &M64 : nullptr, r64.p, x64.p, nk,
                                  std::min(par.restart, par.max_iter - iters), 0.0, abstol_dev.p, true, host_flags,
                                  st);
      }
    } else {
      set_abstol();
      if (compact)
        for (int i = 0; i < na; ++i)
          launch_convert<double, float>(r64.p + (size_t)act[i] * n, r32.p + (size_t)i * n, n, st);
      else
        launch_convert<double, float>(r64.p, r32.p, (long)nrhs * n, st);
      launch_fill_zero(e32.p, (size_t)cur_n * n * sizeof(cplx<float>), st);
      it = krylov_cycle<float>(k32, A32, use_m ? &M32 : nullptr, r32.p, e32.p, na,
                               std::min(par.restart, par.max_iter - iters), 0.0, abstol_dev.p, true, host_flags, st);
      if (compact)
        for (int i = 0; i < na; ++i)
          launch_add_to64<float>(e32.p + (size_t)i * n, x64.p + (size_t)act[i] * n, n, st);
      else
        launch_add_to64<float>(e32.p, x64.p, (long)nrhs * n, st);
    }
    cur_n = nrhs;
    cur_mu = mu_d;
    iters += it;
    cycles += 1;
    // reliable update: r = b - D x in FP64
    launch_dslash<double>(o64, x64.p, t64.p, nrhs, mu_d, st);
    if (nd) launch_flavour_couple<double>(x64.p, t64.p, -eps, n, st);
    launch_xmy<double>(b64.p, t64.p, (long)nrhs * n, st);
    std::swap(r64.p, t64.p);
    if (it == 0 && cycles > 3) break;   // no progress possible
  }
  HIPCHK(hipGetLastError());
  if (info) {
    info->status = status;
    info->outer_iters += iters;
    info->cycles += cycles;
    info->true_rel_resid = std::max(info->true_rel_resid, worst);
  }
  return status;
}

// End of a solve: the coarse-level counters go into info; a persistent
// kernel's barrier wait that gave up turns the status into TMAMG_EHIP (the
// FP64 residual in info still describes x) and retires those kernels for
// the rest of the context.
tmamg_status Ctx::finish(tmamg_info& loc, tmamg_status s) {
  const HierBase::Counters k = hier->take_counters();
  loc.l2_iters_total += k.l2;
  loc.coarsest_iters_total += k.coarsest;
  if (timer.on)
    timer.report("solve", st, " level1_iters=" + std::to_string(k.l2) + " coarsest_iters=" +
                                  std::to_string(k.coarsest) + " coarsest_calls=" + std::to_string(k.coarsest_calls) +
                                  " coarsest_reorth=" + std::to_string(k.reorth));
  if (k.timeouts > 0) {
    hier->disable_persistent();
    g_last_error = "a persistent coarse kernel's barrier wait timed out (" + std::to_string(k.timeouts) +
                   "); the coarsest level uses the generic kernels from now on";
    return TMAMG_EHIP;
  }
  return s;
}

tmamg_status Ctx::solve(const cplx<double>* b, cplx<double>* x, int nrhs, const double* mu_host, double tol,
                        tmamg_info* info, bool guess) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "solve before setup"};
  check(b && x && nrhs >= 1, "bad solve arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  auto t0 = clk::now();
  ensure(nrhs);
  tmamg_info loc{};
  launch_spinor_to_internal<double>(fg, b, b64.p, nrhs, st);
  if (guess) launch_spinor_to_internal<double>(fg, x, x64.p, nrhs, st);
  tmamg_status s = solve_core(nrhs, mu_host, tol, &loc, nullptr, guess);
  launch_spinor_to_canonical<double>(fg, x64.p, x, nrhs, st);
  HIPCHK(hipStreamSynchronize(st));
  s = finish(loc, s);
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

// (D D^dag + sigma) x = b as D(mu') w = b, then x = Gamma5 D(-mu')^-1 Gamma5 w
// (mu' = sqrt(mu^2 + sigma)).  Each solve meets tol on its own system; the
// residual of the product system can still exceed tol by up to
// ||D|| / mu', so it is computed in FP64 and, while above tol, the pair of
// solves is repeated on it and the correction added.
tmamg_status Ctx::solve_shifted(const cplx<double>* b, cplx<double>* x, int nrhs, const double* sigma, double tol,
                                tmamg_info* info) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "solve before setup"};
  check(b && x && sigma && nrhs >= 1, "bad solve arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  auto t0 = clk::now();
  ensure(nrhs);
  const long n = 12 * fg.V;
  const size_t cnt = (size_t)nrhs * n;
  std::vector<double> mup(nrhs), mum(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    check(std::isfinite(sigma[r]) && sigma[r] >= 0, "sigma must be finite and >= 0");
    mup[r] = std::sqrt(mu * mu + sigma[r]);
    mum[r] = -mup[r];
  }
  sh_b.alloc(std::max(sh_b.n, cnt));
  sh_x.alloc(std::max(sh_x.n, cnt));
  tmamg_info loc{};
  launch_spinor_to_internal<double>(fg, b, sh_b.p, nrhs, st);
  std::vector<double> bn = norms(sh_b.p, nrhs);
  launch_fill_zero(sh_x.p, cnt * sizeof(cplx<double>), st);
  HIPCHK(hipMemcpyAsync(b64.p, sh_b.p, cnt * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  const FineOp<double> o64 = op64();
  tmamg_status s = TMAMG_OK;
  double worst = 0;
  for (int pass = 0;; ++pass) {
    // b64 holds the right-hand side of this pass (b, then the product residual)
    tmamg_status s1 = solve_core(nrhs, mup.data(), tol, &loc);
    launch_gamma5_fine<double>(fg, x64.p, b64.p, nrhs, st);
    tmamg_status s2 = solve_core(nrhs, mum.data(), tol, &loc);
    launch_gamma5_fine<double>(fg, x64.p, t64.p, nrhs, st);
    launch_axpby<double>(t64.p, sh_x.p, 1.0, 1.0, (long)cnt, st);
    if (s1 != TMAMG_OK || s2 != TMAMG_OK) s = TMAMG_NOT_CONVERGED;
    // r = b - D(mu') Gamma5 D(-mu') Gamma5 x
    upload_mu(nrhs, mum.data());
    launch_gamma5_fine<double>(fg, sh_x.p, t64.p, nrhs, st);
    launch_dslash<double>(o64, t64.p, r64.p, nrhs, mu_dev.p, st);
    launch_gamma5_fine<double>(fg, r64.p, t64.p, nrhs, st);
    upload_mu(nrhs, mup.data());
    launch_dslash<double>(o64, t64.p, b64.p, nrhs, mu_dev.p, st);
    launch_xmy<double>(sh_b.p, b64.p, (long)cnt, st);
    std::vector<double> rn = norms(b64.p, nrhs);
    worst = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(rn[r])) throw TmError{TMAMG_ENUMERIC, "residual became NaN/Inf"};
      worst = std::max(worst, bn[r] > 0 ? rn[r] / bn[r] : 0.0);
    }
    if (worst <= tol || s != TMAMG_OK || pass == 2) break;
  }
  if (worst > tol) s = TMAMG_NOT_CONVERGED;
  launch_spinor_to_canonical<double>(fg, sh_x.p, x, nrhs, st);
  HIPCHK(hipStreamSynchronize(st));
  s = finish(loc, s);
  loc.true_rel_resid = worst;
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

std::vector<double> Ctx::shifted_residual(const cplx<double>* b, const cplx<double>* x, cplx<double>* r, int nrhs,
                                          const std::vector<double>& mup, const std::vector<double>& bn) {
  const long n = 12 * fg.V;
  std::vector<double> mum(nrhs);
  for (int k = 0; k < nrhs; ++k) mum[k] = -mup[k];
  const FineOp<double> o64 = op64();
  // r = b - D(mu') Gamma5 D(-mu') Gamma5 x
  upload_mu(nrhs, mum.data());
  launch_gamma5_fine<double>(fg, x, t64.p, nrhs, st);
  launch_dslash<double>(o64, t64.p, r64.p, nrhs, mu_dev.p, st);
  launch_gamma5_fine<double>(fg, r64.p, t64.p, nrhs, st);
  upload_mu(nrhs, mup.data());
  launch_dslash<double>(o64, t64.p, r, nrhs, mu_dev.p, st);
  launch_xmy<double>(b, r, (long)nrhs * n, st);
  std::vector<double> rn = norms(r, nrhs);
  for (int k = 0; k < nrhs; ++k) {
    if (!std::isfinite(rn[k])) throw TmError{TMAMG_ENUMERIC, "residual became NaN/Inf"};
    rn[k] = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
  }
  return rn;
}

// Shifted systems (D D^dag + sigma_k) x_k = b of one source with a
// first-order initial guess (Sec. 3, Eq. (6)).  With Q = Gamma5 D(0)
// Hermitian, D D^dag + sigma = Gamma5 (Q + i mu')(Q - i mu') Gamma5, so the two
// solves of a shift are w = (Q + i mu')^-1 Gamma5 b = D(mu')^-1 b and
// u = (Q - i mu')^-1 w = D(-mu')^-1 Gamma5 w, x = Gamma5 u.  Around the base
// shift (the smallest; A = Q + i mu_b, B = Q - i mu_b, delta = mu' - mu_b):
//   w ~ w_b - i delta y_b,         y_b = A^-1 w_b = D(mu_b)^-1 Gamma5 w_b,
//   u ~ u_b + i delta v_b,         v_b = B^-1 (u_b - y_b) = D(-mu_b)^-1 Gamma5 (u_b - y_b),
// the expansion (Q +- i delta)^-1 ~ Q^-1 -+ i delta Q^-2 applied to each
// factor.  The base shift costs four solves (w_b; y_b and u_b as one batch;
// v_b), the others start their two batched solves from these guesses (a
// right-hand side whose guess is worse than zero starts from zero).  The
// shifted systems' own FP64 residuals are then corrected as in
// solve_shifted.
tmamg_status Ctx::solve_multishift(const cplx<double>* b, cplx<double>* x, int nshift, const double* sigma,
                                   double tol, tmamg_info* info) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "solve before setup"};
  check(b && x && sigma && nshift >= 1, "bad solve arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  auto t0 = clk::now();
  ensure(std::max(nshift, 2));
  const long n = 12 * fg.V;
  int base = 0;
  std::vector<double> mup(nshift);
  for (int k = 0; k < nshift; ++k) {
    check(std::isfinite(sigma[k]) && sigma[k] >= 0, "sigma must be finite and >= 0");
    mup[k] = std::sqrt(mu * mu + sigma[k]);
    if (sigma[k] < sigma[base]) base = k;
  }
  const double mb = mup[base];
  const size_t cnt = (size_t)nshift * n, f = n * sizeof(cplx<double>);
  sh_b.alloc(std::max(sh_b.n, cnt));
  sh_x.alloc(std::max(sh_x.n, cnt));
  ms_base.alloc(std::max(ms_base.n, (size_t)4 * n));
  cplx<double>* W = ms_base.p;
  cplx<double>* Y = W + n;
  cplx<double>* U = W + 2 * n;
  cplx<double>* Vb = W + 3 * n;
  tmamg_info loc{};
  tmamg_status s = TMAMG_OK;
  auto fold = [&](tmamg_status st_) { if (st_ != TMAMG_OK) s = TMAMG_NOT_CONVERGED; };
  // the source, in every shift's slot
  launch_spinor_to_internal<double>(fg, b, sh_b.p, 1, st);
  for (int k = 1; k < nshift; ++k) HIPCHK(hipMemcpyAsync(sh_b.p + k * n, sh_b.p, f, hipMemcpyDeviceToDevice, st));
  const std::vector<double> bn(nshift, norms(sh_b.p, 1)[0]);
  // base: w_b
  HIPCHK(hipMemcpyAsync(b64.p, sh_b.p, f, hipMemcpyDeviceToDevice, st));
  fold(solve_core(1, &mb, tol, &loc));
  HIPCHK(hipMemcpyAsync(W, x64.p, f, hipMemcpyDeviceToDevice, st));
  // y_b and u_b: one batch on Gamma5 w_b with +mu_b and -mu_b
  launch_gamma5_fine<double>(fg, W, b64.p, 1, st);
  HIPCHK(hipMemcpyAsync(b64.p + n, b64.p, f, hipMemcpyDeviceToDevice, st));
  const double pm[2] = {mb, -mb};
  fold(solve_core(2, pm, tol, &loc));
  HIPCHK(hipMemcpyAsync(Y, x64.p, f, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(U, x64.p + n, f, hipMemcpyDeviceToDevice, st));
  launch_gamma5_fine<double>(fg, U, sh_x.p + base * n, 1, st);   // the base shift's solution
  if (nshift > 1) {
    // v_b
    launch_lincomb(U, Y, t64.p, -1.0, 0.0, n, st);
    launch_gamma5_fine<double>(fg, t64.p, b64.p, 1, st);
    const double mm = -mb;
    fold(solve_core(1, &mm, tol, &loc));
    HIPCHK(hipMemcpyAsync(Vb, x64.p, f, hipMemcpyDeviceToDevice, st));
    // the other shifts, batched: step 1 from w_b - i delta y_b
    std::vector<int> idx;
    std::vector<double> mk_, mkm;
    for (int k = 0; k < nshift; ++k)
      if (k != base) {
        idx.push_back(k);
        mk_.push_back(mup[k]);
        mkm.push_back(-mup[k]);
      }
    const int m = (int)idx.size();
    for (int j = 0; j < m; ++j) {
      HIPCHK(hipMemcpyAsync(b64.p + j * n, sh_b.p, f, hipMemcpyDeviceToDevice, st));
      launch_lincomb(W, Y, x64.p + j * n, 0.0, -(mk_[j] - mb), n, st);
    }
    fold(solve_core(m, mk_.data(), tol, &loc, nullptr, true));
    // step 2 from u_b + i delta v_b
    launch_gamma5_fine<double>(fg, x64.p, b64.p, m, st);
    for (int j = 0; j < m; ++j) launch_lincomb(U, Vb, x64.p + j * n, 0.0, mk_[j] - mb, n, st);
    fold(solve_core(m, mkm.data(), tol, &loc, nullptr, true));
    for (int j = 0; j < m; ++j) launch_gamma5_fine<double>(fg, x64.p + j * n, sh_x.p + idx[j] * n, 1, st);
  }
  // the shifted systems' own residuals; defect correction where above tol
  double worst = 0;
  for (int pass = 0;; ++pass) {
    std::vector<double> rel = shifted_residual(sh_b.p, sh_x.p, b64.p, nshift, mup, bn);
    worst = *std::max_element(rel.begin(), rel.end());
    if (worst <= tol || s != TMAMG_OK || pass == 2) break;
    std::vector<double> mm(nshift);
    for (int k = 0; k < nshift; ++k) mm[k] = -mup[k];
    fold(solve_core(nshift, mup.data(), tol, &loc));
    launch_gamma5_fine<double>(fg, x64.p, b64.p, nshift, st);
    fold(solve_core(nshift, mm.data(), tol, &loc));
    launch_gamma5_fine<double>(fg, x64.p, t64.p, nshift, st);
    launch_axpby<double>(t64.p, sh_x.p, 1.0, 1.0, (long)cnt, st);
  }
  if (worst > tol) s = TMAMG_NOT_CONVERGED;
  launch_spinor_to_canonical<double>(fg, sh_x.p, x, nshift, st);
  HIPCHK(hipStreamSynchronize(st));
  s = finish(loc, s);
  loc.true_rel_resid = worst;
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

// The even-odd reduced system D_hat(mu) x_e = b_e (the operator the
// paper's simulations work with, Sec. 1.2): with the odd right-hand side
// zero, the full system D [x_e; x_o] = [b_e; 0] has x_o = -D_oo^-1 D_oe x_e
// and hence D_hat x_e = b_e, so the multigrid solve of the full operator
// solves it.  The reduced residual r_hat = b_e - D_hat x_e differs from the
// full one (r_hat = r_e - D_eo D_oo^-1 r_o), so it is computed in FP64 with
// the Schur operator and, while above tol, the full solve is repeated on it
// (defect correction, at most three passes).
tmamg_status Ctx::solve_eo(const cplx<double>* b, cplx<double>* x, int nrhs, const double* mu_host, double tol,
                           tmamg_info* info) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "solve before setup"};
  check(b && x && nrhs >= 1, "bad solve arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  auto t0 = clk::now();
  ensure(nrhs);
  const long n = 12 * fg.V;
  const size_t cnt = (size_t)nrhs * n;
  std::vector<double> m(nrhs, mu);
  if (mu_host)
    for (int r = 0; r < nrhs; ++r) {
      check(std::isfinite(mu_host[r]), "non-finite twisted mass");
      m[r] = mu_host[r];
    }
  sh_b.alloc(std::max(sh_b.n, cnt));
  sh_x.alloc(std::max(sh_x.n, cnt));
  tmamg_info loc{};
  launch_spinor_to_internal<double>(fg, b, sh_b.p, nrhs, st);
  launch_zero_parity<double>(fg, sh_b.p, nrhs, 1, st);
  const std::vector<double> bn = norms(sh_b.p, nrhs);
  launch_fill_zero(sh_x.p, cnt * sizeof(cplx<double>), st);
  HIPCHK(hipMemcpyAsync(b64.p, sh_b.p, cnt * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  const FineOp<double> o64 = op64();
  tmamg_status s = TMAMG_OK;
  double worst = 0;
  for (int pass = 0;; ++pass) {
    // b64: the even right-hand side of this pass, odd sites zero
    if (solve_core(nrhs, m.data(), 0.25 * tol, &loc) != TMAMG_OK) s = TMAMG_NOT_CONVERGED;
    launch_zero_parity<double>(fg, x64.p, nrhs, 1, st);
    launch_axpby<double>(x64.p, sh_x.p, 1.0, 1.0, (long)cnt, st);
    // r_hat = b_e - D_hat x_e
    upload_mu(nrhs, m.data());
    launch_schur<double>(o64, sh_x.p, t64.p, b64.p, nrhs, mu_dev.p, st);
    launch_xmy<double>(sh_b.p, b64.p, (long)cnt, st);
    std::vector<double> rn = norms(b64.p, nrhs);
    worst = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(rn[r])) throw TmError{TMAMG_ENUMERIC, "residual became NaN/Inf"};
      worst = std::max(worst, bn[r] > 0 ? rn[r] / bn[r] : 0.0);
    }
    if (worst <= tol || s != TMAMG_OK || pass == 2) break;
  }
  if (worst > tol) s = TMAMG_NOT_CONVERGED;
  launch_spinor_to_canonical<double>(fg, sh_x.p, x, nrhs, st);
  HIPCHK(hipStreamSynchronize(st));
  s = finish(loc, s);
  loc.true_rel_resid = worst;
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

tmamg_status Ctx::solve_nd(const cplx<double>* b, cplx<double>* x, double mubar, double epsbar, double tol,
                           tmamg_info* info) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "solve before setup"};
  check(b && x, "bad solve arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  check(std::isfinite(mubar) && std::isfinite(epsbar), "non-finite doublet masses");
  auto t0 = clk::now();
  ensure(2);
  const long n = 12 * fg.V;
  const bool flex = par.nlevels >= 1;
  if (par.precision == TMAMG_FP64)
    KN64.ensure(2 * n, par.restart, 1, flex, st);
  else
    KN32.ensure(2 * n, par.restart, 1, flex, st);
  const double mus[2] = {mubar, -mubar};
  tmamg_info loc{};
  launch_spinor_to_internal<double>(fg, b, b64.p, 2, st);
  tmamg_status s = solve_core(2, mus, tol, &loc, &epsbar);
  launch_spinor_to_canonical<double>(fg, x64.p, x, 2, st);
  HIPCHK(hipStreamSynchronize(st));
  s = finish(loc, s);
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

tmamg_status Ctx::force(const cplx<double>* phi, cplx<double>* F, double* S, double tol, tmamg_info* info,
                        const double* mu_force) {
  if (!have_setup) throw TmError{TMAMG_ESTATE, "force before setup"};
  check(phi && F && S, "bad force arguments");
  check(tol > 0 && tol < 1, "tol must be in (0, 1)");
  auto t0 = clk::now();
  ensure(1);
  tmamg_info loc{};
  const long n = 12 * fg.V;
  const double mf = mu_force ? *mu_force : mu;
  check(std::isfinite(mf), "non-finite twisted mass");
  double mp = mf, mm = -mf;
  // Y = D(mu)^-1 phi
  launch_spinor_to_internal<double>(fg, phi, b64.p, 1, st);
  DevArr<cplx<double>> Y;
  Y.alloc(n);
  tmamg_status s1 = solve_core(1, &mp, tol, &loc);
  HIPCHK(hipMemcpyAsync(Y.p, x64.p, n * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  // X = Gamma5 D(-mu)^-1 Gamma5 Y, in t64 (free once the solves are done)
  launch_gamma5_fine<double>(fg, Y.p, b64.p, 1, st);
  tmamg_status s2 = solve_core(1, &mm, tol, &loc);
  cplx<double>* X = t64.p;
  launch_gamma5_fine<double>(fg, x64.p, X, 1, st);
  // The Krylov bases hold nothing live after the solves: phi (internal
  // layout, n values) and the clover part's field of the force kernels
  // (54 per site) borrow their memory where it is large enough, which keeps
  // the force within the solver's own footprint at large volumes; the
  // borrowed bytes are cleared afterwards (the next solve's bases start
  // from zeros).
  const size_t phi_b = (size_t)n * sizeof(cplx<double>), xi_b = (size_t)54 * fg.V * sizeof(cplx<double>);
  struct Pool { char* p; size_t left; };
  Pool pools[2] = {{nullptr, 0}, {nullptr, 0}};
  if (par.precision == TMAMG_FP64) {
    pools[0] = {reinterpret_cast<char*>(K64.V.p), K64.V.bytes()};
    pools[1] = {reinterpret_cast<char*>(K64.Z.p), K64.Z.bytes()};
  } else {
    pools[0] = {reinterpret_cast<char*>(K32.V.p), K32.V.bytes()};
    pools[1] = {reinterpret_cast<char*>(K32.Z.p), K32.Z.bytes()};
  }
  std::vector<std::pair<char*, size_t>> borrowed;
  DevArr<cplx<double>> own_phi, own_xi;
  auto take = [&](size_t bytes, DevArr<cplx<double>>& own) -> cplx<double>* {
    for (Pool& q : pools)
      if (q.p && q.left >= bytes) {
        char* r = q.p;
        q.p += (bytes + 255) / 256 * 256;
        q.left = q.left > (bytes + 255) / 256 * 256 ? q.left - (bytes + 255) / 256 * 256 : 0;
        borrowed.emplace_back(r, bytes);
        return reinterpret_cast<cplx<double>*>(r);
      }
    own.alloc(bytes / sizeof(cplx<double>));
    return own.p;
  };
  cplx<double>* xi = csw != 0.0 ? take(xi_b, own_xi) : nullptr;
  cplx<double>* phi64 = take(phi_b, own_phi);
  launch_spinor_to_internal<double>(fg, phi, phi64, 1, st);
  // S = Re <phi, X>
  int NB = reduce_blocks(n);
  launch_multidot<double>(phi64, n, 1, X, n, 1, red_partial.p, NB, nullptr, st);
  launch_finalize(red_partial.p, 1, 1, NB, red_out.p, 1, st);
  double sv[2];
  HIPCHK(hipMemcpyAsync(sv, red_out.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  launch_force(op64(), csw, X, Y.p, F, st, xi);
  for (auto& b : borrowed) launch_fill_zero(b.first, b.second, st);
  HIPCHK(hipStreamSynchronize(st));
  *S = sv[0];
  tmamg_status s = (s1 == TMAMG_OK && s2 == TMAMG_OK) ? TMAMG_OK : TMAMG_NOT_CONVERGED;
  s = finish(loc, s);
  loc.t_setup_s = t_setup;
  loc.t_solve_s = std::chrono::duration<double>(clk::now() - t0).count();
  loc.status = s;
  if (info) *info = loc;
  return s;
}

void Ctx::force_link_gradient(const cplx<double>* F, cplx<double>* G, double scale) {
  if (!have_links) throw TmError{TMAMG_ESTATE, "link gradient before setup"};
  check(F && G, "null pointer");
  check(std::isfinite(scale), "scale must be finite");
  launch_link_gradient(op64(), lat.t_antiperiodic, F, G, scale, st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
}

// The same with every intermediate field in the caller-provided device
// workspace ws (78 complex doubles per site: X and Y in the internal layout,
// then the clover part's field); allocates nothing.
void Ctx::force_from_fields_ws(const cplx<double>* X, const cplx<double>* Y, cplx<double>* F, cplx<double>* ws) {
  if (!have_links) throw TmError{TMAMG_ESTATE, "force before setup"};
  check(X && Y && F, "null pointer");
  const long n = 12 * fg.V;
  cplx<double>* Xi = ws;
  cplx<double>* Yi = ws + n;
  launch_spinor_to_internal<double>(fg, X, Xi, 1, st);
  launch_spinor_to_internal<double>(fg, Y, Yi, 1, st);
  launch_force(op64(), csw, Xi, Yi, F, st, ws + 2 * n);
  HIPCHK(hipStreamSynchronize(st));
}

void Ctx::force_from_fields(const cplx<double>* X, const cplx<double>* Y, cplx<double>* F) {
  if (!have_links) throw TmError{TMAMG_ESTATE, "force before setup"};
  check(X && Y && F, "null pointer");
  const long n = 12 * fg.V;
  DevArr<cplx<double>> Xi, Yi;
  Xi.alloc(n);
  Yi.alloc(n);
  launch_spinor_to_internal<double>(fg, X, Xi.p, 1, st);
  launch_spinor_to_internal<double>(fg, Y, Yi.p, 1, st);
  launch_force(op64(), csw, Xi.p, Yi.p, F, st);
  HIPCHK(hipStreamSynchronize(st));
}

void Ctx::apply(int op, int level, const cplx<double>* in, cplx<double>* out, int nrhs, const double* mu_host) {
  check(in && out && nrhs >= 1, "bad apply arguments");
  if (!have_links) throw TmError{TMAMG_ESTATE, "apply before setup"};
  ensure(nrhs);
  upload_mu(nrhs, mu_host);
  const long n0 = 12 * fg.V;
  if (op == TMAMG_OP_DDAG64 || op == TMAMG_OP_DDAG32) {
    // D(mu)^dag = Gamma5 D(-mu) Gamma5
    check(level == 0, "D^dag acts on level 0");
    std::vector<double> neg(nrhs);
    for (int r = 0; r < nrhs; ++r) neg[r] = -(mu_host ? mu_host[r] : mu);
    upload_mu(nrhs, neg.data());
    launch_spinor_to_internal<double>(fg, in, b64.p, nrhs, st);
    launch_gamma5_fine<double>(fg, b64.p, r64.p, nrhs, st);
    if (op == TMAMG_OP_DDAG64) {
      launch_dslash<double>(op64(), r64.p, t64.p, nrhs, mu_dev.p, st);
    } else {
      if (!links32.p) throw TmError{TMAMG_EINVAL, "FP32 operator needs mixed precision"};
      DevArr<cplx<float>> a, b;
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * n0);
      launch_convert<double, float>(r64.p, a.p, (long)nrhs * n0, st);
      launch_dslash<float>(op32(), a.p, b.p, nrhs, mu_dev.p, st);
      launch_convert<float, double>(b.p, t64.p, (long)nrhs * n0, st);
      HIPCHK(hipStreamSynchronize(st));
    }
    launch_gamma5_fine<double>(fg, t64.p, b64.p, nrhs, st);
    launch_spinor_to_canonical<double>(fg, b64.p, out, nrhs, st);
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
  if (op == TMAMG_OP_D64 || op == TMAMG_OP_D32 || op == TMAMG_OP_SCHUR64 || op == TMAMG_OP_SCHUR32) {
    check(level == 0, "D acts on level 0");
    launch_spinor_to_internal<double>(fg, in, b64.p, nrhs, st);
    if (op == TMAMG_OP_D64) {
      launch_dslash<double>(op64(), b64.p, t64.p, nrhs, mu_dev.p, st);
    } else if (op == TMAMG_OP_SCHUR64) {
      launch_schur<double>(op64(), b64.p, r64.p, t64.p, nrhs, mu_dev.p, st);
    } else if (op == TMAMG_OP_SCHUR32) {
      if (!links32.p) throw TmError{TMAMG_EINVAL, "FP32 operator needs mixed precision"};
      DevArr<cplx<float>> a, b, c;
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * n0);
      c.alloc((size_t)nrhs * n0);
      launch_convert<double, float>(b64.p, a.p, (long)nrhs * n0, st);
      launch_schur<float>(op32(), a.p, c.p, b.p, nrhs, mu_dev.p, st);
      launch_convert<float, double>(b.p, t64.p, (long)nrhs * n0, st);
      HIPCHK(hipStreamSynchronize(st));
    } else {
      if (!links32.p) throw TmError{TMAMG_EINVAL, "FP32 operator needs mixed precision"};
      DevArr<cplx<float>> a, b;
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * n0);
      launch_convert<double, float>(b64.p, a.p, (long)nrhs * n0, st);
      launch_dslash<float>(op32(), a.p, b.p, nrhs, mu_dev.p, st);
      launch_convert<float, double>(b.p, t64.p, (long)nrhs * n0, st);
      HIPCHK(hipStreamSynchronize(st));
    }
    launch_spinor_to_canonical<double>(fg, t64.p, out, nrhs, st);
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
  if (!have_setup) throw TmError{TMAMG_ESTATE, "hierarchy not set up"};
  double dc_eps = 0.0;
  if (op == TMAMG_OP_DCND || op == TMAMG_OP_SAPND) {
    check(nrhs == 2 && mu_host != nullptr, "the doublet operators take two flavours and {mubar, epsbar}");
    check(std::isfinite(mu_host[0]) && std::isfinite(mu_host[1]), "non-finite doublet masses");
    const double m2[2] = {mu_host[0], -mu_host[0]};
    upload_mu(2, m2);
    dc_eps = mu_host[1];
  }
  struct EpsScope {
    HierBase* h;
    EpsScope(HierBase* h_, double e) : h(h_) { h->nd_eps = e; }
    ~EpsScope() { h->nd_eps = 0.0; }
  } eps_scope(hier.get(), dc_eps);
  long sites_in, sites_out;
  int dof_in, dof_out;
  int lin = level, lout = level;
  if (op == TMAMG_OP_PROLONG) lout = level - 1;
  if (op == TMAMG_OP_RESTRICT) lout = level + 1;
  check(lin >= 0 && lin <= 2 && lout >= 0 && lout <= 2, "bad level");
  tmamg_level_info(reinterpret_cast<const tmamg_ctx*>(this), lin, &sites_in, &dof_in);
  tmamg_level_info(reinterpret_cast<const tmamg_ctx*>(this), lout, &sites_out, &dof_out);
  check(sites_in > 0 && sites_out > 0, "level not present");
  const long nin = sites_in * dof_in * nrhs, nout = sites_out * dof_out * nrhs;
  DevArr<cplx<double>> i64, o64;
  i64.alloc(nin);
  o64.alloc(nout);
  if (lin == 0) launch_spinor_to_internal<double>(fg, in, i64.p, nrhs, st);
  else HIPCHK(hipMemcpyAsync(i64.p, in, nin * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  if (hier->is_double()) {
    hier->test_op(op, level, i64.p, o64.p, nrhs, mu_dev.p);
  } else {
    DevArr<cplx<float>> i32, o32;
    i32.alloc(nin);
    o32.alloc(nout);
    launch_convert<double, float>(i64.p, i32.p, nin, st);
    hier->test_op(op, level, i32.p, o32.p, nrhs, mu_dev.p);
    launch_convert<float, double>(o32.p, o64.p, nout, st);
    HIPCHK(hipStreamSynchronize(st));
  }
  if (lout == 0) launch_spinor_to_canonical<double>(fg, o64.p, out, nrhs, st);
  else HIPCHK(hipMemcpyAsync(out, o64.p, nout * sizeof(cplx<double>), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  (void)drain_counters();
}

double Ctx::time_kernel(int kernel, int nrhs, int reps) {
  check(nrhs >= 1 && reps >= 1, "nrhs and reps must be positive");
  if (!have_links) throw TmError{TMAMG_ESTATE, "timing before setup"};
  // the stencil timings use buffers of their own: the solve workspace
  // (sized for nrhs with its Krylov bases) is not grown for a measurement
  const long n0 = 12 * fg.V;
  if (kernel == TMAMG_K_DSLASH64 || kernel == TMAMG_K_DSLASH32) {
    DevArr<double> mu_t;
    mu_t.alloc(nrhs);
    hipLaunchKernelGGL(k_fill_double, dim3((nrhs + 63) / 64), dim3(64), 0, st, mu_t.p, mu, nrhs);
    if (kernel == TMAMG_K_DSLASH64) {
      DevArr<cplx<double>> a, b;
      a.alloc((size_t)nrhs * n0);
      b.alloc((size_t)nrhs * n0);
      launch_random<double>(a.p, (long)nrhs * n0, 21, st);
      FineOp<double> o = op64();
      return time_launches(st, reps, [&]() { launch_dslash<double>(o, a.p, b.p, nrhs, mu_t.p, st); });
    }
    if (!links32.p) throw TmError{TMAMG_EINVAL, "FP32 operator needs mixed precision"};
    DevArr<cplx<float>> a, b;
    a.alloc((size_t)nrhs * n0);
    b.alloc((size_t)nrhs * n0);
    launch_random<float>(a.p, (long)nrhs * n0, 22, st);
    FineOp<float> o = op32();
    return time_launches(st, reps, [&]() { launch_dslash<float>(o, a.p, b.p, nrhs, mu_t.p, st); });
  }
  if (kernel == TMAMG_K_SCHUR32) {
    if (!links32.p) throw TmError{TMAMG_EINVAL, "FP32 operator needs mixed precision"};
    DevArr<double> mu_t;
    mu_t.alloc(nrhs);
    hipLaunchKernelGGL(k_fill_double, dim3((nrhs + 63) / 64), dim3(64), 0, st, mu_t.p, mu, nrhs);
    DevArr<cplx<float>> a, b, t;
    a.alloc((size_t)nrhs * n0);
    b.alloc((size_t)nrhs * n0);
    t.alloc((size_t)nrhs * n0);
    launch_random<float>(a.p, (long)nrhs * n0, 23, st);
    FineOp<float> o = op32();
    return time_launches(st, reps, [&]() { launch_schur<float>(o, a.p, t.p, b.p, nrhs, mu_t.p, st); });
  }
  if (kernel == TMAMG_K_COPY) {
    const size_t bytes = (size_t)512 << 20;
    DevArr<unsigned char> a, b;
    a.alloc(bytes);
    b.alloc(bytes);
    launch_fill_zero(a.p, bytes, st);
    return time_launches(st, reps, [&]() { launch_copy16(a.p, b.p, bytes, st); });
  }
  if (!have_setup) throw TmError{TMAMG_ESTATE, "timing before setup"};
  return hier->time_kernel(kernel, nrhs, reps);
}

// Autotuner: for each family with more than one kernel for the
// hierarchy's shapes, force each variant in turn, time it with HIP events
// on the hierarchy's own operators (the same launches as time_kernel), and
// keep the fastest in the variant table with every variant's time.  A
// variant the launcher did not run (not available for this precision,
// storage or shape) is not a candidate; a shape with no candidate gets no
// entry.
template <typename T, typename S>
void Hier<T, S>::autotune(int nrhs, int reps) {
  struct Job { int fam, kernel; long a, b; };
  std::vector<Job> jobs;
  jobs.push_back({TUNE_SAP0, TMAMG_K_SAP0, c->fg.bvol, c->fg.V});
  if (nlev >= 2) {
    jobs.push_back({TUNE_RESTRICT0, TMAMG_K_RESTRICT0, nv0, c->fg.V});
    jobs.push_back({TUNE_PROLONG0, TMAMG_K_PROLONG0, nv0, c->fg.V});
    jobs.push_back({TUNE_COARSE_APPLY, TMAMG_K_DC1, d1, g1.V});
  }
  if (nlev >= 3) {
    jobs.push_back({TUNE_COARSE_APPLY, TMAMG_K_DC2, d2, g2.V});
    jobs.push_back({TUNE_SAP1, TMAMG_K_SAP1, d1, g1.V});
  }
  for (const Job& j : jobs) {
    double ms[TUNE_MAX_VARIANTS] = {-1.0, -1.0, -1.0, -1.0};
    const int nvar = tune_variants(j.fam);
    int best = -1;
    for (int v = 0; v < nvar; ++v) {
      tune_put(j.fam, j.a, j.b, nrhs, v, nullptr, 0);
      tune_used(j.fam, -1);
      const double t = time_kernel(j.kernel, nrhs, reps);
      if (tune_last_used(j.fam) != v) continue;
      ms[v] = t;
      if (best < 0 || t < ms[best]) best = v;
    }
    tune_put(j.fam, j.a, j.b, nrhs, best, ms, nvar);
  }
}

void Ctx::autotune(const int* nrhs_list, int n, int reps) {
  check(nrhs_list != nullptr && n >= 1 && reps >= 1, "autotune needs right-hand-side counts and reps >= 1");
  for (int k = 0; k < n; ++k) check(nrhs_list[k] >= 1 && nrhs_list[k] <= 64, "right-hand-side counts must be 1..64");
  if (!have_setup) throw TmError{TMAMG_ESTATE, "autotune before setup"};
  for (int k = 0; k < n; ++k) hier->autotune(nrhs_list[k], reps);
  HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ allocation-free scratch
// Device scratch of tmamg_force_from_fields_noalloc: a file-scope device
// array (every GPU the library runs on holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: it
// stands for no device address on the host.  The device address of each
// GPU's copy is taken once per device, with that device current, when the
// first context is created on it, and only that address is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)160 << 20;
constexpr size_t NOALLOC_BYTES_PER_SITE = 78 * sizeof(cplx<double>);
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[256];

static void* device_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) throw TmError{TMAMG_EHIP, "device index out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw TmError{TMAMG_EHIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e)};
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// ------------------------------------------------------------------ C ABI
template <typename F>
static tmamg_status guarded(F&& f) {
  try {
    return f();
  } catch (const TmError& e) {
    g_last_error = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return TMAMG_EINVAL;
  }
}

static Ctx* C(tmamg_ctx* c) { return reinterpret_cast<Ctx*>(c); }
static const Ctx* C(const tmamg_ctx* c) { return reinterpret_cast<const Ctx*>(c); }

// An entry point on a context: errors become statuses, and every device
// buffer the call allocates comes from the context's allocator.
template <typename F>
static tmamg_status with_ctx(tmamg_ctx* ctx, F&& f) {
  return guarded([&]() -> tmamg_status {
    check(ctx != nullptr, "null context");
    Ctx* c = C(ctx);
    AllocScope scope(&c->dalloc);
    return f(c);
  });
}

extern "C" {

tmamg_status tmamg_default_params(tmamg_params* p) {
  if (!p) { g_last_error = "null params"; return TMAMG_EINVAL; }
  std::memset(p, 0, sizeof(*p));
  p->nlevels = 2;
  for (int m = 0; m < 4; ++m) { p->agg[0][m] = 4; p->agg[1][m] = 2; p->sap_block1[m] = 2; }
  p->nv[0] = 12;
  p->nv[1] = 32;
  p->setup_iters = 3;
  p->init_smooth = 2;
  p->sap_sweeps[0] = 4;
  p->sap_sweeps[1] = 2;
  p->mr_steps = 4;
  p->l2_iters = 10;
  p->l2_tol = 0.1;
  p->coarsest_iters = 100;
  p->coarsest_tol = 0.1;
  p->restart = 30;
  p->max_iter = 2000;
  p->precision = TMAMG_FP64;
  p->storage = TMAMG_STORE_BF16;
  p->inner_tol = 1e-3;
  p->seed = 4001;
  p->nd_coarse_coupling = 1;
  p->setup_chunk = 0;
  p->keep_test_vectors = 1;
  return TMAMG_OK;
}

tmamg_status tmamg_create(tmamg_ctx** ctx, const tmamg_lattice* lat, const tmamg_params* par, void* hip_stream,
                          const tmamg_allocator* allocator) {
  return guarded([&]() {
    check(ctx && lat && par, "null argument");
    *ctx = nullptr;
    std::unique_ptr<Ctx> c(new Ctx(*lat, *par, reinterpret_cast<hipStream_t>(hip_stream), allocator));
    c->scratch = device_scratch();
    *ctx = reinterpret_cast<tmamg_ctx*>(c.release());
    return TMAMG_OK;
  });
}

tmamg_status tmamg_setup(tmamg_ctx* ctx, const void* U, double kappa, double csw, double mu) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->setup(static_cast<const cplx<double>*>(U), kappa, csw, mu);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_setup_update(tmamg_ctx* ctx, const void* U, int iters) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->setup_update(static_cast<const cplx<double>*>(U), iters);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_solve(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                         tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, mu_rhs, tol,
                         info);
  });
}

tmamg_status tmamg_solve_guess(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                               tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, mu_rhs, tol, info,
                    true);
  });
}

tmamg_status tmamg_debug_inject(tmamg_ctx* ctx, int what) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(what == 0, "what must be 0 (barrier timeout)");
    if (!c->have_setup || c->par.nlevels < 2) throw TmError{TMAMG_ESTATE, "needs a multigrid setup"};
    c->hier->flag_barrier_timeout();
    return TMAMG_OK;
  });
}

tmamg_status tmamg_solve_shifted(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* sigma, double tol,
                                 tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve_shifted(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, sigma,
                                 tol, info);
  });
}

tmamg_status tmamg_solve_eo(tmamg_ctx* ctx, const void* b, void* x, int nrhs, const double* mu_rhs, double tol,
                            tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve_eo(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, mu_rhs, tol, info);
  });
}

tmamg_status tmamg_solve_multishift(tmamg_ctx* ctx, const void* b, void* x, int nshift, const double* sigma,
                                    double tol, tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve_multishift(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nshift, sigma,
                               tol, info);
  });
}

tmamg_status tmamg_solve_nd(tmamg_ctx* ctx, const void* b, void* x, double mubar, double epsbar, double tol,
                            tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->solve_nd(static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), mubar, epsbar, tol,
                            info);
  });
}

tmamg_status tmamg_force(tmamg_ctx* ctx, const void* phi, void* F, double* S, double tol, tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->force(static_cast<const cplx<double>*>(phi), static_cast<cplx<double>*>(F), S, tol, info);
  });
}

tmamg_status tmamg_force_at(tmamg_ctx* ctx, const void* phi, double mu, void* F, double* S, double tol,
                            tmamg_info* info) {
  return with_ctx(ctx, [&](Ctx* c) {
    return c->force(static_cast<const cplx<double>*>(phi), static_cast<cplx<double>*>(F), S, tol, info, &mu);
  });
}

tmamg_status tmamg_gauge_force(tmamg_ctx* ctx, const void* U, double beta, void* F, double* S) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(U && F && S, "null argument");
    check(std::isfinite(beta), "beta must be finite");
    *S = md_gauge_force(c->lat, static_cast<const cplx<double>*>(U), beta, static_cast<cplx<double>*>(F), c->st);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_md_update_links(tmamg_ctx* ctx, void* U, const void* P, double eps) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(U && P, "null argument");
    check(std::isfinite(eps), "eps must be finite");
    md_update_links(c->lat, static_cast<cplx<double>*>(U), static_cast<const cplx<double>*>(P), eps, c->st);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_md_update_momenta(tmamg_ctx* ctx, void* P, const void* F, double coef) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(P && F, "null argument");
    check(std::isfinite(coef), "coef must be finite");
    md_update_momenta(c->lat, static_cast<cplx<double>*>(P), static_cast<const cplx<double>*>(F), coef, c->st);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_md_kinetic(tmamg_ctx* ctx, const void* P, double* K) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(P && K, "null argument");
    *K = md_kinetic(c->lat, static_cast<const cplx<double>*>(P), c->st);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_force_link_gradient(tmamg_ctx* ctx, const void* F, void* G, double scale) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->force_link_gradient(static_cast<const cplx<double>*>(F), static_cast<cplx<double>*>(G), scale);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_force_from_fields(tmamg_ctx* ctx, const void* X, const void* Y, void* F) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->force_from_fields(static_cast<const cplx<double>*>(X), static_cast<const cplx<double>*>(Y),
                              static_cast<cplx<double>*>(F));
    return TMAMG_OK;
  });
}

tmamg_status tmamg_force_from_fields_noalloc(tmamg_ctx* ctx, const void* X, const void* Y, void* F) {
  return with_ctx(ctx, [&](Ctx* c) {
    const size_t need = (size_t)c->fg.V * NOALLOC_BYTES_PER_SITE;
    if (need > NOALLOC_SCRATCH_BYTES)
      throw TmError{TMAMG_EINVAL, "the allocation-free force needs " + std::to_string(need) +
                                      " bytes of scratch (78 complex doubles per site); its static array holds " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES) + " (at most " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES / NOALLOC_BYTES_PER_SITE) + " sites)"};
    c->force_from_fields_ws(static_cast<const cplx<double>*>(X), static_cast<const cplx<double>*>(Y),
                            static_cast<cplx<double>*>(F), static_cast<cplx<double>*>(c->scratch));
    return TMAMG_OK;
  });
}

tmamg_status tmamg_apply(tmamg_ctx* ctx, int op, int level, const void* in, void* out, int nrhs,
                         const double* mu_rhs) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->apply(op, level, static_cast<const cplx<double>*>(in), static_cast<cplx<double>*>(out), nrhs, mu_rhs);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_debug_set_test_vectors(tmamg_ctx* ctx, int level, const void* v) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(v != nullptr, "null argument");
    check(level == 0 || level == 1, "test vectors live on level 0 or 1");
    check(c->par.nlevels >= level + 2, "no such coarsening");
    if (level == 0) {
      long n = 12 * c->fg.V;
      c->inject0.alloc((size_t)c->par.nv[0] * n);
      launch_spinor_to_internal<double>(c->fg, static_cast<const cplx<double>*>(v), c->inject0.p, c->par.nv[0], c->st);
    } else {
      long n = (long)c->fg.nblocks * 2 * c->par.nv[0];
      c->inject1.alloc((size_t)c->par.nv[1] * n);
      HIPCHK(hipMemcpyAsync(c->inject1.p, v, c->par.nv[1] * n * sizeof(cplx<double>), hipMemcpyDeviceToDevice, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    return TMAMG_OK;
  });
}

tmamg_status tmamg_debug_export(tmamg_ctx* ctx, int what, int level, void* out) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(out != nullptr, "null argument");
    if (!c->have_setup) throw TmError{TMAMG_ESTATE, "export before setup"};
    if (what == 0) c->hier->export_P(level, static_cast<cplx<double>*>(out));
    else if (what == 1) c->hier->export_Dc(level, static_cast<cplx<double>*>(out));
    else throw TmError{TMAMG_EINVAL, "what must be 0 (P) or 1 (D_c)"};
    HIPCHK(hipStreamSynchronize(c->st));
    return TMAMG_OK;
  });
}

tmamg_status tmamg_level_info(const tmamg_ctx* ctx, int level, long* sites, int* dof) {
  return guarded([&]() {
    check(ctx && sites && dof, "null argument");
    const Ctx* c = C(ctx);
    *sites = 0;
    *dof = 0;
    if (level == 0) { *sites = c->fg.V; *dof = 12; }
    else if (level == 1 && c->par.nlevels >= 2) { *sites = c->fg.nblocks; *dof = 2 * c->par.nv[0]; }
    else if (level == 2 && c->par.nlevels >= 3) {
      long s = 1;
      for (int m = 0; m < 4; ++m) s *= c->fg.NB[m] / c->par.agg[1][m];
      *sites = s;
      *dof = 2 * c->par.nv[1];
    } else throw TmError{TMAMG_EINVAL, "no such level"};
    return TMAMG_OK;
  });
}

tmamg_status tmamg_time_kernel(tmamg_ctx* ctx, int kernel, int nrhs, int reps, double* avg_ms) {
  return with_ctx(ctx, [&](Ctx* c) {
    check(avg_ms != nullptr, "null argument");
    *avg_ms = c->time_kernel(kernel, nrhs, reps);
    return TMAMG_OK;
  });
}

tmamg_status tmamg_autotune(tmamg_ctx* ctx, const int* nrhs_list, int n, int reps, const char* json_path) {
  return with_ctx(ctx, [&](Ctx* c) {
    c->autotune(nrhs_list, n, reps);
    if (json_path) {
      int dev = 0;
      hipDeviceProp_t prop;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipGetDeviceProperties(&prop, dev));
      check(tune_save(json_path, prop.gcnArchName), "cannot write the tuning file");
    }
    return TMAMG_OK;
  });
}

tmamg_status tmamg_tune_load(const char* json_path, int* n_entries) {
  return guarded([&]() {
    check(json_path != nullptr, "null path");
    const int n = tune_load(json_path);
    check(n >= 0, "unreadable or malformed tuning file");
    if (n_entries) *n_entries = n;
    return TMAMG_OK;
  });
}

tmamg_status tmamg_tune_save(const char* json_path) {
  return guarded([&]() {
    check(json_path != nullptr, "null path");
    check(tune_save(json_path, ""), "cannot write the tuning file");
    return TMAMG_OK;
  });
}

tmamg_status tmamg_tune_set(int family, long a, long b, long nrhs, int variant) {
  return guarded([&]() {
    check(family >= 0 && family < TUNE_NFAM, "unknown kernel family");
    check(variant >= -1 && variant < tune_variants(family), "variant out of range for this family");
    tune_put(family, a, b, nrhs, variant, nullptr, 0);
    return TMAMG_OK;
  });
}

int tmamg_tune_get(int family, long a, long b, long nrhs) { return tune_get(family, a, b, nrhs); }

int tmamg_tune_entries(void) { return tune_entries(); }

void tmamg_tune_clear(void) { tune_clear(); }

void tmamg_destroy(tmamg_ctx* ctx) {
  try {
    delete C(ctx);
  } catch (...) {
  }
}

const char* tmamg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
