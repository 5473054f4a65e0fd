// Pseudofermion force of S_f = phi^dag (D D^dag)^-1 phi (K13-K15).
//
// With Y = D^-1 phi and X = (D D^dag)^-1 phi, dS = -2 Re <X, dD Y>.  For a
// variation U_l(z) -> exp(w) U_l(z), w in su(3), dS = Re tr(w M) with
//   hopping:  M = U Lam1 - Lam2 U^dag,
//             Lam1 = sum_{ss'} (1 - g_l)_{ss'} Y_s'(z+l) X_s(z)^dag,
//             Lam2 = sum_{ss'} (1 + g_l)_{ss'} Y_s'(z) X_s(z+l)^dag;
//   clover:   dS = Re sum_x sum_{mu<nu} tr(dQ_{mu nu}(x) Xi_{mu nu}(x)),
//             Xi = -(i c_sw / 8) (Sig' + Sig'^dag), Sig' the traceless part of
//             Sig_{mu nu}(x) = sum_{ss'} (sigma_{mu nu})_{ss'} Y_s'(x) X_s(x)^dag;
//             each plaquette holding the link contributes, for each of its
//             four corners c, the closed path from the link with Xi(c)
//             inserted where the path passes c (with a minus sign and the
//             path starting after the link when the link is traversed
//             backwards).
// The force is F = -1/2 TA(M), TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6, so that
// dS/dt = -2 tr(F w) with generators T^a = i lambda^a / 2.
// Links are the internal ones (time-boundary sign folded in); the sign
// cancels in M.
#include "solver.h"
#include "su3.h"

struct SigmaTab {
  double re[6][2][2][2];
  double im[6][2][2][2];
};

__device__ long site_shift(const FineGeom& g, const int c[4], int m1, int s1, int m2 = 0, int s2 = 0) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  if (s1) cc[m1] = (cc[m1] + s1 + g.L[m1]) % g.L[m1];
  if (s2) cc[m2] = (cc[m2] + s2 + g.L[m2]) % g.L[m2];
  return fine_index(g, cc);
}

__device__ int plane_index(int a, int b) {
  // (0,1)=0 (0,2)=1 (0,3)=2 (1,2)=3 (1,3)=4 (2,3)=5
  return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

__global__ void k_force_xi(FineGeom g, SigmaTab sg, double csw, const cplx<double>* __restrict__ X,
                           const cplx<double>* __restrict__ Y, cplx<double>* Xi) {
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  cplx<double> x[12], y[12];
  const size_t ts = tsite((unsigned)s, 12);
  for (int k = 0; k < 12; ++k) { x[k] = X[ts + k * FT]; y[k] = Y[ts + k * FT]; }
  for (int p = 0; p < 6; ++p) {
    cplx<double> S[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[i][j] = mk(0.0, 0.0);
    for (int ch = 0; ch < 2; ++ch)
      for (int a = 0; a < 2; ++a)       // spin s = 2ch + a (row of sigma)
        for (int b = 0; b < 2; ++b) {   // spin s' = 2ch + b
          cplx<double> sv = mk(sg.re[p][ch][a][b], sg.im[p][ch][a][b]);
          if (sv.re == 0 && sv.im == 0) continue;
          const cplx<double>* ys = y + (2 * ch + b) * 3;
          const cplx<double>* xs = x + (2 * ch + a) * 3;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S[i][j] += sv * (ys[i] * conj(xs[j]));
        }
    cplx<double> tr = (1.0 / 3.0) * (S[0][0] + S[1][1] + S[2][2]);
    for (int i = 0; i < 3; ++i) S[i][i] -= tr;
    // Xi = -(i csw/8) (S + S^dag)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cplx<double> h = S[i][j] + conj(S[j][i]);
        cplx<double> v = (-csw / 8.0) * times_i(h);
        Xi[((long)p * 9 + i * 3 + j) * g.V + s] = v;
      }
  }
}

__device__ M3<double> load_xi(const cplx<double>* Xi, int p, long s, long V) {
  M3<double> m;
  for (int k = 0; k < 9; ++k) m.e[k / 3][k % 3] = Xi[((long)p * 9 + k) * V + s];
  return m;
}

__device__ M3<double> m3_scale_add(const M3<double>& a, const M3<double>& b, double sb) {
  M3<double> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.e[i][j] = a.e[i][j] + sb * b.e[i][j];
  return r;
}

// sum over corners: W0..W3 the closed path; Xa[k] the Xi at the corner reached after step k+1.
// forward: Xi of the start corner (= Xa[3]) goes at the end; backward: Xs at the start, negated.
__device__ M3<double> insert_sum(const M3<double> W[4], const M3<double> Xa[4], bool backward) {
  M3<double> p1 = W[0];
  M3<double> p2 = m3_mul(p1, W[1]);
  M3<double> p3 = m3_mul(p2, W[2]);
  M3<double> p4 = m3_mul(p3, W[3]);
  M3<double> s3 = W[3];
  M3<double> s2 = m3_mul(W[2], W[3]);
  M3<double> s1 = m3_mul(W[1], s2);
  M3<double> r = backward ? m3_mul(Xa[3], p4) : m3_mul(p4, Xa[3]);
  r = m3_add(r, m3_mul(m3_mul(p1, Xa[0]), s1));
  r = m3_add(r, m3_mul(m3_mul(p2, Xa[1]), s2));
  r = m3_add(r, m3_mul(m3_mul(p3, Xa[2]), s3));
  if (backward) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) r.e[i][j] = -r.e[i][j];
  }
  return r;
}

template <int L>
__device__ void hop_lambda(const FineOp<double>& op, const cplx<double>* X, const cplx<double>* Y, long z, long zp,
                           cplx<double> L1[3][3], cplx<double> L2[3][3]) {
  const long V = op.g.V;
  cplx<double> yn[12], xz[12], yz[12], xn[12];
  const size_t tz = tsite((unsigned)z, 12), tp = tsite((unsigned)zp, 12);
  for (int k = 0; k < 12; ++k) {
    yn[k] = Y[tp + k * FT];
    xz[k] = X[tz + k * FT];
    yz[k] = Y[tz + k * FT];
    xn[k] = X[tp + k * FT];
  }
  // (1 - g) Y(z+l) and (1 + g) Y(z) as full spinors via the chiral projection
  cplx<double> h[6], pm[12], pp[12];
  project<L, -1>(yn, h);
  for (int c = 0; c < 3; ++c) {
    pm[c] = h[c];
    pm[3 + c] = h[3 + c];
    cplx<double> a0, a1;
    mulAdag<L>(h[c], h[3 + c], a0, a1);
    pm[6 + c] = -a0;
    pm[9 + c] = -a1;
  }
  project<L, +1>(yz, h);
  for (int c = 0; c < 3; ++c) {
    pp[c] = h[c];
    pp[3 + c] = h[3 + c];
    cplx<double> a0, a1;
    mulAdag<L>(h[c], h[3 + c], a0, a1);
    pp[6 + c] = a0;
    pp[9 + c] = a1;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> a = mk(0.0, 0.0), b = mk(0.0, 0.0);
      for (int sp = 0; sp < 4; ++sp) {
        a += pm[sp * 3 + i] * conj(xz[sp * 3 + j]);
        b += pp[sp * 3 + i] * conj(xn[sp * 3 + j]);
      }
      L1[i][j] = a;
      L2[i][j] = b;
    }
}

__global__ void k_force_links(FineOp<double> op, const cplx<double>* __restrict__ X, const cplx<double>* __restrict__ Y,
                              const cplx<double>* __restrict__ Xi, int with_clover, cplx<double>* F) {
  const FineGeom& g = op.g;
  long z = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (z >= g.V) return;
  const int lam = blockIdx.y;
  const long V = g.V;
  int c[4];
  fine_coords(g, z, c);
  long zp = site_shift(g, c, lam, 1);
  M3<double> U = load_link(op.links, lam, z, V);
  cplx<double> L1[3][3], L2[3][3];
  switch (lam) {
    case 0: hop_lambda<0>(op, X, Y, z, zp, L1, L2); break;
    case 1: hop_lambda<1>(op, X, Y, z, zp, L1, L2); break;
    case 2: hop_lambda<2>(op, X, Y, z, zp, L1, L2); break;
    default: hop_lambda<3>(op, X, Y, z, zp, L1, L2); break;
  }
  M3<double> A1, A2;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { A1.e[i][j] = L1[i][j]; A2.e[i][j] = L2[i][j]; }
  M3<double> M = m3_scale_add(m3_mul(U, A1), m3_mul_ad(A2, U), -1.0);
  if (with_clover) {
    for (int nu = 0; nu < 4; ++nu) {
      if (nu == lam) continue;
      const int a = lam < nu ? lam : nu, b = lam < nu ? nu : lam;
      const int p = plane_index(a, b);
      M3<double> W[4], Xa[4];
      if (lam == a) {
        // P1: forward as the first leg of P(z; a, b)
        W[0] = U;
        W[1] = load_link(op.links, b, site_shift(g, c, a, 1), V);
        W[2] = m3_dag(load_link(op.links, a, site_shift(g, c, b, 1), V));
        W[3] = m3_dag(load_link(op.links, b, z, V));
        Xa[0] = load_xi(Xi, p, site_shift(g, c, a, 1), V);
        Xa[1] = load_xi(Xi, p, site_shift(g, c, a, 1, b, 1), V);
        Xa[2] = load_xi(Xi, p, site_shift(g, c, b, 1), V);
        Xa[3] = load_xi(Xi, p, z, V);
        M = m3_add(M, insert_sum(W, Xa, false));
        // P2: backward as the third leg of P(z - b; a, b)
        long y = site_shift(g, c, b, -1);
        W[0] = m3_dag(load_link(op.links, b, y, V));
        W[1] = load_link(op.links, a, y, V);
        W[2] = load_link(op.links, b, site_shift(g, c, b, -1, a, 1), V);
        W[3] = m3_dag(U);
        Xa[0] = load_xi(Xi, p, y, V);
        Xa[1] = load_xi(Xi, p, site_shift(g, c, b, -1, a, 1), V);
        Xa[2] = load_xi(Xi, p, site_shift(g, c, a, 1), V);
        Xa[3] = load_xi(Xi, p, z, V);
        M = m3_add(M, insert_sum(W, Xa, true));
      } else {
        // P3: forward as the second leg of P(z - a; a, b)
        long y = site_shift(g, c, a, -1);
        W[0] = U;
        W[1] = m3_dag(load_link(op.links, a, site_shift(g, c, a, -1, b, 1), V));
        W[2] = m3_dag(load_link(op.links, b, y, V));
        W[3] = load_link(op.links, a, y, V);
        Xa[0] = load_xi(Xi, p, site_shift(g, c, b, 1), V);
        Xa[1] = load_xi(Xi, p, site_shift(g, c, a, -1, b, 1), V);
        Xa[2] = load_xi(Xi, p, y, V);
        Xa[3] = load_xi(Xi, p, z, V);
        M = m3_add(M, insert_sum(W, Xa, false));
        // P4: backward as the fourth leg of P(z; a, b)
        W[0] = load_link(op.links, a, z, V);
        W[1] = load_link(op.links, b, site_shift(g, c, a, 1), V);
        W[2] = m3_dag(load_link(op.links, a, site_shift(g, c, b, 1), V));
        W[3] = m3_dag(U);
        Xa[0] = load_xi(Xi, p, site_shift(g, c, a, 1), V);
        Xa[1] = load_xi(Xi, p, site_shift(g, c, a, 1, b, 1), V);
        Xa[2] = load_xi(Xi, p, site_shift(g, c, b, 1), V);
        Xa[3] = load_xi(Xi, p, z, V);
        M = m3_add(M, insert_sum(W, Xa, true));
      }
    }
  }
  // F = -1/2 TA(M)
  cplx<double> A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (M.e[i][j] - conj(M.e[j][i]));
  cplx<double> tr = (1.0 / 3.0) * (A[0][0] + A[1][1] + A[2][2]);
  for (int i = 0; i < 3; ++i) A[i][i] -= tr;
  // canonical output index
  long cs = ((long)(c[3] * g.L[2] + c[2]) * g.L[1] + c[1]) * g.L[0] + c[0];
  cplx<double>* out = F + ((long)lam * V + cs) * 9;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i * 3 + j] = -0.5 * A[i][j];
}

void sigma_blocks(double re[6][2][2][2], double im[6][2][2][2]);

void launch_force(const FineOp<double>& op, double csw, const cplx<double>* X, const cplx<double>* Y,
                  cplx<double>* F_canon, hipStream_t st, cplx<double>* xi_ws) {
  SigmaTab sg;
  sigma_blocks(sg.re, sg.im);
  DevArr<cplx<double>> Xi;
  const bool clover = csw != 0.0;
  cplx<double>* xi = xi_ws;
  if (clover) {
    if (!xi) {
      Xi.alloc((size_t)6 * 9 * op.g.V);
      xi = Xi.p;
    }
    hipLaunchKernelGGL(k_force_xi, dim3((unsigned)((op.g.V + 127) / 128)), dim3(128), 0, st, op.g, sg, csw, X, Y,
                       xi);
  }
  hipLaunchKernelGGL(k_force_links, dim3((unsigned)((op.g.V + 127) / 128), 4), dim3(128), 0, st, op, X, Y,
                     clover ? xi : nullptr, clover ? 1 : 0, F_canon);
  HIPCHK(hipStreamSynchronize(st));
}

// Link gradient for automatic differentiation: G_mu(x) = 2 scale F_mu(x) U_mu(x)
// with the caller's links U (internal links carry the time-boundary sign,
// undone here), canonical layout in and out.  For U -> exp(X) U with X in
// su(3), Re sum conj(G) (X U) = -2 scale tr(F X) = scale dS/dt: G is the
// complex gradient dS/dRe U + i dS/dIm U on the directions tangent to SU(3).
__global__ void k_link_gradient(FineGeom g, const cplx<double>* __restrict__ links, int antiperiodic,
                                const cplx<double>* __restrict__ F, cplx<double>* __restrict__ G, double scale) {
  const long cs = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (cs >= g.V) return;
  const int mu = blockIdx.y;
  int c[4];
  long r = cs;
  c[0] = (int)(r % g.L[0]); r /= g.L[0];
  c[1] = (int)(r % g.L[1]); r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
  const double sign = (antiperiodic && mu == 3 && c[3] == g.L[3] - 1) ? -1.0 : 1.0;
  const M3<double> U = load_link(links, mu, fine_index(g, c), g.V);
  const cplx<double>* f = F + ((long)mu * g.V + cs) * 9;
  cplx<double>* o = G + ((long)mu * g.V + cs) * 9;
  const double k = 2.0 * sign * scale;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx<double> acc = f[i * 3] * U.e[0][j];
      cfma(acc, f[i * 3 + 1], U.e[1][j]);
      cfma(acc, f[i * 3 + 2], U.e[2][j]);
      o[i * 3 + j] = k * acc;
    }
}

void launch_link_gradient(const FineOp<double>& op, int antiperiodic, const cplx<double>* F_canon,
                          cplx<double>* G_canon, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_link_gradient, dim3((unsigned)((op.g.V + 127) / 128), 4), dim3(128), 0, st, op.g, op.links,
                     antiperiodic, F_canon, G_canon, scale);
}
