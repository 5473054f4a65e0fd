// Molecular-dynamics pieces of the (mini) HMC of Sec. 2: the Wilson
// plaquette gauge action and its force (innermost time scale of the nested
// integrator), the momentum and link updates and the kinetic energy.  All
// fields are in the canonical layout [4][T][Z][Y][X][3][3] (complex128),
// the gauge field periodic in every direction.
#include "solver.h"

namespace {

struct Lat4 {
  int L[4];
  long V;
};

TM_D long site_shift(const Lat4& g, long s, int mu, int step) {
  long st = 1;
  for (int m = 0; m < mu; ++m) st *= g.L[m];
  const int c = (int)((s / st) % g.L[mu]);
  const int cn = (c + step + g.L[mu]) % g.L[mu];
  return s + (long)(cn - c) * st;
}

TM_D void ld(const cplx<double>* U, int mu, long s, long V, cplx<double> m[3][3]) {
  const cplx<double>* p = U + ((long)mu * V + s) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k / 3][k % 3] = p[k];
}
// c = a b, c = a b^dag, c = a^dag b
TM_D void mm(const cplx<double> a[3][3], const cplx<double> b[3][3], cplx<double> c[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> t = a[i][0] * b[0][j];
      cfma(t, a[i][1], b[1][j]);
      cfma(t, a[i][2], b[2][j]);
      c[i][j] = t;
    }
}
TM_D void mmd(const cplx<double> a[3][3], const cplx<double> b[3][3], cplx<double> c[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> t = a[i][0] * conj(b[j][0]);
      cfma(t, a[i][1], conj(b[j][1]));
      cfma(t, a[i][2], conj(b[j][2]));
      c[i][j] = t;
    }
}
TM_D void mdm(const cplx<double> a[3][3], const cplx<double> b[3][3], cplx<double> c[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> t = cmulc(a[0][i], b[0][j]);
      cfmac(t, a[1][i], b[1][j]);
      cfmac(t, a[2][i], b[2][j]);
      c[i][j] = t;
    }
}

// Block sums of per-thread values into part[blockIdx] (256 threads).
TM_D void block_sum_to(double v, double* part) {
  __shared__ double red[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Force on U_mu(x): with the staples S = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag +
// U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)], dS_g/dt = -(beta/3) Re tr(w U S), so
// F = (beta/6) TA(U S).  Also the plaquette sum: the thread of (x, mu) adds
// Re tr P_{mu nu}(x) for nu > mu.
__global__ void __launch_bounds__(256) k_gauge_force(Lat4 g, const cplx<double>* __restrict__ U, double beta,
                                                      cplx<double>* __restrict__ F, double* part) {
  const long s = blockIdx.x * 256L + threadIdx.x;
  const int mu = blockIdx.y;
  double plaq = 0;
  if (s < g.V) {
    cplx<double> S[3][3], a[3][3], b[3][3], c[3][3], t[3][3], u[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[i][j] = mk(0.0, 0.0);
    const long xp = site_shift(g, s, mu, 1);
    ld(U, mu, s, g.V, u);
    for (int nu = 0; nu < 4; ++nu) {
      if (nu == mu) continue;
      // forward staple
      ld(U, nu, xp, g.V, a);
      ld(U, mu, site_shift(g, s, nu, 1), g.V, b);
      ld(U, nu, s, g.V, c);
      mmd(a, b, t);
      mmd(t, c, a);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[i][j] += a[i][j];
      if (nu > mu) {
        // Re tr (U_mu(x) * forward staple) is the plaquette P_{mu nu}(x)
        mm(u, a, t);
        plaq += t[0][0].re + t[1][1].re + t[2][2].re;
      }
      // backward staple
      const long xm = site_shift(g, s, nu, -1);
      ld(U, nu, site_shift(g, xp, nu, -1), g.V, a);
      ld(U, mu, xm, g.V, b);
      ld(U, nu, xm, g.V, c);
      // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag = (U_mu(x-nu) U_nu(x+mu-nu))^dag
      mm(b, a, t);
      mdm(t, c, a);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[i][j] += a[i][j];
    }
    mm(u, S, t);
    // TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6
    cplx<double> tr = mk(0.0, 0.0);
    for (int i = 0; i < 3; ++i) tr += t[i][i] - conj(t[i][i]);
    cplx<double>* o = F + ((long)mu * g.V + s) * 9;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cplx<double> v = 0.5 * (t[i][j] - conj(t[j][i]));
        if (i == j) v -= (1.0 / 6.0) * tr;
        o[i * 3 + j] = (beta / 6.0) * v;
      }
  }
  block_sum_to(plaq, part);
}

// U <- exp(eps P) U: scaling and squaring of a Taylor series (degree 10 on
// a matrix of norm <= 1/4), per link
__global__ void __launch_bounds__(256) k_md_links(long n, cplx<double>* __restrict__ U,
                                                   const cplx<double>* __restrict__ P, double eps) {
  const long l = blockIdx.x * 256L + threadIdx.x;
  if (l >= n) return;
  cplx<double> A[3][3], E[3][3], T[3][3], u[3][3];
  double nrm = 0;
  for (int i = 0; i < 3; ++i) {
    double row = 0;
    for (int j = 0; j < 3; ++j) {
      A[i][j] = eps * P[l * 9 + i * 3 + j];
      row += sqrt(norm2(A[i][j]));
    }
    nrm = fmax(nrm, row);
  }
  int k = 0;
  while (nrm > 0.25 && k < 40) {
    nrm *= 0.5;
    ++k;
  }
  const double sc = ldexp(1.0, -k);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = sc * A[i][j];
  // Horner: E = I + A (I + A/2 (I + A/3 (... (I + A/10))))
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) E[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int d = 10; d >= 1; --d) {
    mm(A, E, T);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) E[i][j] = (1.0 / d) * T[i][j] + mk(i == j ? 1.0 : 0.0, 0.0);
  }
  for (int q = 0; q < k; ++q) {
    mm(E, E, T);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) E[i][j] = T[i][j];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) u[i][j] = U[l * 9 + i * 3 + j];
  mm(E, u, T);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U[l * 9 + i * 3 + j] = T[i][j];
}

__global__ void k_md_axpy(long n, cplx<double>* __restrict__ P, const cplx<double>* __restrict__ F, double c) {
  const long k = blockIdx.x * 256L + threadIdx.x;
  if (k < n) P[k] += c * F[k];
}

__global__ void __launch_bounds__(256) k_md_sumsq(long n, const cplx<double>* __restrict__ P, double* part) {
  const long k = blockIdx.x * 256L + threadIdx.x;
  block_sum_to(k < n ? norm2(P[k]) : 0.0, part);
}

double host_sum(const DevArr<double>& part, size_t count, hipStream_t st) {
  std::vector<double> h(count);
  HIPCHK(hipMemcpyAsync(h.data(), part.p, count * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double s = 0;
  for (double v : h) s += v;   // fixed order
  return s;
}

Lat4 lat4(const tmamg_lattice& l) {
  Lat4 g;
  g.V = 1;
  for (int m = 0; m < 4; ++m) {
    g.L[m] = l.dims[m];
    g.V *= l.dims[m];
  }
  return g;
}

}  // namespace

double md_gauge_force(const tmamg_lattice& lat, const cplx<double>* U, double beta, cplx<double>* F, hipStream_t st) {
  const Lat4 g = lat4(lat);
  const unsigned nb = (unsigned)((g.V + 255) / 256);
  DevArr<double> part;
  part.alloc((size_t)nb * 4);
  hipLaunchKernelGGL(k_gauge_force, dim3(nb, 4), dim3(256), 0, st, g, U, beta, F, part.p);
  const double plaq = host_sum(part, (size_t)nb * 4, st);
  return beta * (6.0 * (double)g.V - plaq / 3.0);
}

void md_update_links(const tmamg_lattice& lat, cplx<double>* U, const cplx<double>* P, double eps, hipStream_t st) {
  const long n = 4 * lat4(lat).V;
  hipLaunchKernelGGL(k_md_links, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, U, P, eps);
  HIPCHK(hipStreamSynchronize(st));
}

void md_update_momenta(const tmamg_lattice& lat, cplx<double>* P, const cplx<double>* F, double c, hipStream_t st) {
  const long n = 36 * lat4(lat).V;
  hipLaunchKernelGGL(k_md_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, P, F, c);
  HIPCHK(hipStreamSynchronize(st));
}

double md_kinetic(const tmamg_lattice& lat, const cplx<double>* P, hipStream_t st) {
  const long n = 36 * lat4(lat).V;
  const unsigned nb = (unsigned)((n + 255) / 256);
  DevArr<double> part;
  part.alloc(nb);
  hipLaunchKernelGGL(k_md_sumsq, dim3(nb), dim3(256), 0, st, n, P, part.p);
  return host_sum(part, nb, st);
}
