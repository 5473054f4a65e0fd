// 3x3 complex matrices, the chiral spin projection of the hopping term and
// the packed clover block product.
#pragma once

#include "common.h"

template <typename T>
struct M3 {
  cplx<T> e[3][3];
};

template <typename T> TM_HD M3<T> m3_mul(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<T> s = a.e[i][0] * b.e[0][j];
      cfma(s, a.e[i][1], b.e[1][j]);
      cfma(s, a.e[i][2], b.e[2][j]);
      r.e[i][j] = s;
    }
  return r;
}
// a * b^dag
template <typename T> TM_HD M3<T> m3_mul_ad(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<T> s = a.e[i][0] * conj(b.e[j][0]);
      cfma(s, a.e[i][1], conj(b.e[j][1]));
      cfma(s, a.e[i][2], conj(b.e[j][2]));
      r.e[i][j] = s;
    }
  return r;
}
// a^dag * b
template <typename T> TM_HD M3<T> m3_mul_da(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<T> s = cmulc(a.e[0][i], b.e[0][j]);
      cfmac(s, a.e[1][i], b.e[1][j]);
      cfmac(s, a.e[2][i], b.e[2][j]);
      r.e[i][j] = s;
    }
  return r;
}
template <typename T> TM_HD M3<T> m3_dag(const M3<T>& a) {
  M3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = conj(a.e[j][i]);
  return r;
}
template <typename T> TM_HD M3<T> m3_add(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[i][j] = a.e[i][j] + b.e[i][j];
  return r;
}

// U_mu(s): links are four tiled 9-component arrays, one per direction.
template <typename T>
TM_D M3<T> load_link(const cplx<T>* __restrict__ links, int mu, long s, long V) {
  M3<T> u;
  const cplx<T>* p = links + (size_t)mu * 9 * V + tsite((unsigned)s, 9);
#pragma unroll
  for (int k = 0; k < 9; ++k) u.e[k / 3][k % 3] = p[k * FT];
  return u;
}
template <int MU, typename T>
TM_D M3<T> load_link_u(const cplx<T>* __restrict__ links, unsigned s, long V) {
  return load_link(links, MU, s, V);
}

// Streaming loads (non-temporal hint) for data used once per kernel, so it
// does not push out of L2 what neighbouring workgroups still read.
template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T> TM_D cplx<T> ld_stream(const cplx<T>* p) {
  const typename Vec2<T>::type v = __builtin_nontemporal_load(reinterpret_cast<const typename Vec2<T>::type*>(p));
  return mk<T>(v.x, v.y);
}
template <typename T> TM_D void st_stream(cplx<T>* p, cplx<T> v) {
  typename Vec2<T>::type x;
  x.x = v.re;
  x.y = v.im;
  __builtin_nontemporal_store(x, reinterpret_cast<typename Vec2<T>::type*>(p));
}
template <int MU, typename T>
TM_D M3<T> load_link_stream(const cplx<T>* __restrict__ links, unsigned s, long V) {
  M3<T> u;
  const cplx<T>* p = links + (size_t)MU * 9 * V + tsite(s, 9);
#pragma unroll
  for (int k = 0; k < 9; ++k) u.e[k / 3][k % 3] = ld_stream(p + k * FT);
  return u;
}

// w = U h (colour), h a colour vector
template <typename T> TM_D void su3_mv(const M3<T>& u, const cplx<T>* h, cplx<T>* w) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cplx<T> s = u.e[i][0] * h[0];
    cfma(s, u.e[i][1], h[1]);
    cfma(s, u.e[i][2], h[2]);
    w[i] = s;
  }
}
// w = U^dag h
template <typename T> TM_D void su3_dmv(const M3<T>& u, const cplx<T>* h, cplx<T>* w) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cplx<T> s = cmulc(u.e[0][i], h[0]);
    cfmac(s, u.e[1][i], h[1]);
    cfmac(s, u.e[2][i], h[2]);
    w[i] = s;
  }
}

// Chiral basis: g_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = -i sigma_k, A_t = 1.
// Spinor index = spin*3 + colour; spins 0,1 are the upper (chirality +) half.
//
// (1 - g_mu) psi = (h ; -A^dag h) with h = u - A d
// (1 + g_mu) psi = (h ;  A^dag h) with h = u + A d
template <int MU, typename T> TM_D void mulA(cplx<T> d0, cplx<T> d1, cplx<T>& o0, cplx<T>& o1) {
  if constexpr (MU == 0) { o0 = -times_i(d1); o1 = -times_i(d0); }       // -i s1
  else if constexpr (MU == 1) { o0 = -d1; o1 = d0; }                      // -i s2
  else if constexpr (MU == 2) { o0 = -times_i(d0); o1 = times_i(d1); }    // -i s3
  else { o0 = d0; o1 = d1; }
}
template <int MU, typename T> TM_D void mulAdag(cplx<T> w0, cplx<T> w1, cplx<T>& o0, cplx<T>& o1) {
  if constexpr (MU == 0) { o0 = times_i(w1); o1 = times_i(w0); }
  else if constexpr (MU == 1) { o0 = w1; o1 = -w0; }
  else if constexpr (MU == 2) { o0 = times_i(w0); o1 = -times_i(w1); }
  else { o0 = w0; o1 = w1; }
}

// h (2 spins x 3 colours) = u + SGN * A d
template <int MU, int SGN, typename T> TM_D void project(const cplx<T>* p, cplx<T>* h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<T> a0, a1;
    mulA<MU>(p[6 + c], p[9 + c], a0, a1);
    if constexpr (SGN > 0) { h[c] = p[c] + a0; h[3 + c] = p[3 + c] + a1; }
    else { h[c] = p[c] - a0; h[3 + c] = p[3 + c] - a1; }
  }
}

// acc += -1/2 (1 -/+ g_mu) reconstructed from w = U h:
//   forward (1 - g): upper += -w/2, lower += +A^dag w/2
//   backward (1 + g): upper += -w/2, lower += -A^dag w/2
template <int MU, int SGN, typename T> TM_D void reconstruct(const cplx<T>* w, cplx<T>* acc) {
  const T half = (T)0.5;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[c] -= half * w[c];
    acc[3 + c] -= half * w[3 + c];
    cplx<T> a0, a1;
    mulAdag<MU>(w[c], w[3 + c], a0, a1);
    if constexpr (SGN > 0) { acc[6 + c] -= half * a0; acc[9 + c] -= half * a1; }
    else { acc[6 + c] += half * a0; acc[9 + c] += half * a1; }
  }
}

// forward hop: acc += -1/2 (1 - g_mu) U_mu(x) psi(x+mu)
template <int MU, typename T> TM_D void hop_fwd(const M3<T>& u, const cplx<T>* pn, cplx<T>* acc) {
  cplx<T> h[6], w[6];
  project<MU, -1>(pn, h);
  su3_mv(u, h, w);
  su3_mv(u, h + 3, w + 3);
  reconstruct<MU, -1>(w, acc);
}
// backward hop: acc += -1/2 (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
template <int MU, typename T> TM_D void hop_bwd(const M3<T>& u, const cplx<T>* pn, cplx<T>* acc) {
  cplx<T> h[6], w[6];
  project<MU, +1>(pn, h);
  su3_dmv(u, h, w);
  su3_dmv(u, h + 3, w + 3);
  reconstruct<MU, +1>(w, acc);
}

// Packed Hermitian 6x6: 6 real diagonal, then upper (i<j) row-major, 15 complex.
TM_HD int herm_idx(int i, int j) { return i * 6 - i * (i + 1) / 2 + (j - i - 1); }

// acc[0..5] += A v[0..5]; cl is one chirality's tiled 36-component array
template <typename T, bool STREAM = false>
TM_D void clover_block_mv(const T* __restrict__ cl, unsigned s, long V, const cplx<T>* v, cplx<T>* acc) {
  T a[36];
  const T* p = cl + tsite(s, 36);
#pragma unroll
  for (int k = 0; k < 36; ++k) a[k] = STREAM ? __builtin_nontemporal_load(p + k * FT) : p[k * FT];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    cplx<T> row = acc[i];
    row.re = fmaT(a[i], v[i].re, row.re);
    row.im = fmaT(a[i], v[i].im, row.im);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j == i) continue;
      if (j > i) {
        int k = 6 + 2 * herm_idx(i, j);
        cfma(row, mk(a[k], a[k + 1]), v[j]);
      } else {
        int k = 6 + 2 * herm_idx(j, i);
        cfmac(row, mk(a[k], a[k + 1]), v[j]);
      }
    }
    acc[i] = row;
  }
}

// Compiler-only fence (emits no instruction): memory accesses may not move
// across it and the accumulator must be fully computed at this point, so
// each hopping direction's loads and arithmetic stay together.
template <typename T>
TM_D void compiler_fence(cplx<T>* acc) {
#pragma unroll
  for (int k = 0; k < 12; ++k) __asm__ __volatile__("" : "+v"(acc[k].re), "+v"(acc[k].im));
  __asm__ __volatile__("" ::: "memory");
}

