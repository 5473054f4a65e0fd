// Shared device/host definitions for the twisted-mass DD-alpha-AMG library.
//
// Complex arithmetic on (re, im) pairs, storage conversions (fp64, fp32,
// bf16, fp16 with round-to-nearest-even), and the block-major site
// ordering of the fine lattice.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>

#define TM_HD __host__ __device__ __forceinline__
#define TM_D __device__ __forceinline__

// ------------------------------------------------------------------ complex
template <typename T>
struct __align__(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T> TM_HD cplx<T> mk(T r, T i) { cplx<T> c; c.re = r; c.im = i; return c; }
template <typename T> TM_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> TM_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> TM_HD cplx<T> operator-(cplx<T> a) { return mk(-a.re, -a.im); }
template <typename T> TM_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> TM_HD cplx<T> operator*(T s, cplx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T> TM_HD cplx<T>& operator+=(cplx<T>& a, cplx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T> TM_HD cplx<T>& operator-=(cplx<T>& a, cplx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T> TM_HD cplx<T> conj(cplx<T> a) { return mk(a.re, -a.im); }
// conj(a) * b
template <typename T> TM_HD cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// Accumulations are written as explicit chains of fused multiply-adds
// (four per complex product): written as a += (x*y - u*v) the compiler may
// only fuse one of the products and then adds, three instructions per real
// component instead of two.
TM_HD float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
TM_HD double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a += b * c
template <typename T> TM_HD void cfma(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fmaT(b.re, c.re, a.re);
  a.re = fmaT(-b.im, c.im, a.re);
  a.im = fmaT(b.re, c.im, a.im);
  a.im = fmaT(b.im, c.re, a.im);
}
// a += conj(b) * c
template <typename T> TM_HD void cfmac(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fmaT(b.re, c.re, a.re);
  a.re = fmaT(b.im, c.im, a.re);
  a.im = fmaT(b.re, c.im, a.im);
  a.im = fmaT(-b.im, c.re, a.im);
}
// a -= b * c
template <typename T> TM_HD void cfms(cplx<T>& a, cplx<T> b, cplx<T> c) {
  a.re = fmaT(-b.re, c.re, a.re);
  a.re = fmaT(b.im, c.im, a.re);
  a.im = fmaT(-b.re, c.im, a.im);
  a.im = fmaT(-b.im, c.re, a.im);
}
// s += |a|^2
template <typename T> TM_HD void acc_norm2(T& s, cplx<T> a) {
  s = fmaT(a.re, a.re, s);
  s = fmaT(a.im, a.im, s);
}
// (sre, sim) += conj(a) * b
template <typename T> TM_HD void acc_dotc(T& sre, T& sim, cplx<T> a, cplx<T> b) {
  sre = fmaT(a.re, b.re, sre);
  sre = fmaT(a.im, b.im, sre);
  sim = fmaT(a.re, b.im, sim);
  sim = fmaT(-a.im, b.re, sim);
}
template <typename T> TM_HD cplx<T> times_i(cplx<T> a) { return mk(-a.im, a.re); }
template <typename T> TM_HD T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------------ storage
// A complex number stored in precision S and computed with in precision T.
template <typename S> struct Store;
template <> struct Store<double> {
  using pair = cplx<double>;
  template <typename T> TM_D static cplx<T> cvt(pair v) { return mk<T>((T)v.re, (T)v.im); }
  template <typename T> TM_D static cplx<T> ld(const pair* p) { pair v = *p; return mk<T>((T)v.re, (T)v.im); }
  template <typename T> TM_D static void st(pair* p, cplx<T> v) { *p = mk<double>((double)v.re, (double)v.im); }
};
template <> struct Store<float> {
  using pair = cplx<float>;
  template <typename T> TM_D static cplx<T> cvt(pair v) { return mk<T>((T)v.re, (T)v.im); }
  template <typename T> TM_D static cplx<T> ld(const pair* p) { pair v = *p; return mk<T>((T)v.re, (T)v.im); }
  template <typename T> TM_D static void st(pair* p, cplx<T> v) { *p = mk<float>((float)v.re, (float)v.im); }
};
struct __align__(4) bf16pair { __hip_bfloat16 re, im; };
struct __align__(4) halfpair { __half re, im; };
template <> struct Store<__hip_bfloat16> {
  using pair = bf16pair;
  template <typename T> TM_D static cplx<T> cvt(pair v) {
    return mk<T>((T)__bfloat162float(v.re), (T)__bfloat162float(v.im));
  }
  template <typename T> TM_D static cplx<T> ld(const pair* p) {
    pair v = *p;
    return mk<T>((T)__bfloat162float(v.re), (T)__bfloat162float(v.im));
  }
  template <typename T> TM_D static void st(pair* p, cplx<T> v) {
    pair o;
    o.re = __float2bfloat16((float)v.re);   // round to nearest even
    o.im = __float2bfloat16((float)v.im);
    *p = o;
  }
};
template <> struct Store<__half> {
  using pair = halfpair;
  template <typename T> TM_D static cplx<T> cvt(pair v) { return mk<T>((T)__half2float(v.re), (T)__half2float(v.im)); }
  template <typename T> TM_D static cplx<T> ld(const pair* p) {
    pair v = *p;
    return mk<T>((T)__half2float(v.re), (T)__half2float(v.im));
  }
  template <typename T> TM_D static void st(pair* p, cplx<T> v) {
    pair o;
    o.re = __float2half((float)v.re);
    o.im = __float2half((float)v.im);
    *p = o;
  }
};

// Four consecutive stored complex numbers, loaded with one vector access.
template <typename S>
struct __align__(4 * sizeof(typename Store<S>::pair)) Quad {
  typename Store<S>::pair e[4];
};

// ------------------------------------------------------------------ fine geometry
// Sites are stored block-major: the lattice is cut into blocks of shape
// B[0..3] (the level-1 aggregate, which is also the SAP block); sites of a
// block are contiguous, x fastest inside the block, and blocks are ordered
// lexicographically (x fastest).  Block b is coarse site b.
struct FineGeom {
  int L[4];       // lattice extents x, y, z, t
  int B[4];       // block extents
  int NB[4];      // blocks per dimension
  int lstride[4]; // stride of a local coordinate inside a block
  int bstride[4]; // stride of a block coordinate (in blocks)
  int bvol;       // sites per block
  int nblocks;
  long V;
};

TM_HD void fine_coords(const FineGeom& g, long s, int c[4]) {
  int b = (int)(s / g.bvol);
  int l = (int)(s - (long)b * g.bvol);
  int lc0 = l % g.B[0]; l /= g.B[0];
  int lc1 = l % g.B[1]; l /= g.B[1];
  int lc2 = l % g.B[2];
  int lc3 = l / g.B[2];
  int b0 = b % g.NB[0]; b /= g.NB[0];
  int b1 = b % g.NB[1]; b /= g.NB[1];
  int b2 = b % g.NB[2];
  int b3 = b / g.NB[2];
  c[0] = b0 * g.B[0] + lc0;
  c[1] = b1 * g.B[1] + lc1;
  c[2] = b2 * g.B[2] + lc2;
  c[3] = b3 * g.B[3] + lc3;
}

TM_HD long fine_index(const FineGeom& g, const int c[4]) {
  int b = 0, l = 0;
  for (int m = 3; m >= 0; --m) {
    b = b * g.NB[m] + c[m] / g.B[m];
    l = l * g.B[m] + c[m] % g.B[m];
  }
  return (long)b * g.bvol + l;
}

// Neighbour of site s (coordinates c) in direction mu, step +1 or -1, periodic.
TM_HD long fine_neighbour(const FineGeom& g, long s, const int c[4], int mu, int step) {
  int lc = c[mu] % g.B[mu];
  int bc = c[mu] / g.B[mu];
  if (step > 0) {
    if (lc < g.B[mu] - 1) return s + g.lstride[mu];
    long ds = -(long)(g.B[mu] - 1) * g.lstride[mu];
    long db = (bc < g.NB[mu] - 1) ? g.bstride[mu] : -(long)(g.NB[mu] - 1) * g.bstride[mu];
    return s + ds + db * g.bvol;
  } else {
    if (lc > 0) return s - g.lstride[mu];
    long ds = (long)(g.B[mu] - 1) * g.lstride[mu];
    long db = (bc > 0) ? -(long)g.bstride[mu] : (long)(g.NB[mu] - 1) * g.bstride[mu];
    return s + ds + db * g.bvol;
  }
}

// Fine-lattice arrays are tiled: FT consecutive sites (in the block-major
// order above) form a tile, and a tile stores its NC components one after
// the other, FT sites each.  Element (s, k) of an NC-component array sits
// at tsite(s, NC) + k * FT.  A wave then reads one component of 64
// consecutive sites as contiguous memory, and all components of one site
// hang off a single address with small immediate offsets.
constexpr unsigned FT = 32;
TM_HD size_t tsite(unsigned s, unsigned nc) { return (size_t)(s / FT) * nc * FT + (s % FT); }

// ------------------------------------------------------------------ coarse geometry
// Coarse lattices are lexicographic (x fastest) and periodic.
struct CoarseGeom {
  int L[4];
  long V;
};

TM_HD void coarse_coords(const CoarseGeom& g, long s, int c[4]) {
  long r = s;
  c[0] = (int)(r % g.L[0]); r /= g.L[0];
  c[1] = (int)(r % g.L[1]); r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
}
TM_HD long coarse_index(const CoarseGeom& g, const int c[4]) {
  return ((long)(c[3] * g.L[2] + c[2]) * g.L[1] + c[1]) * g.L[0] + c[0];
}
TM_HD long coarse_neighbour(const CoarseGeom& g, const int c[4], int mu, int step) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  cc[mu] = (cc[mu] + step + g.L[mu]) % g.L[mu];
  return coarse_index(g, cc);
}

// Scalar-coordinate variants (no runtime-indexed private arrays, which the
// compiler would place in scratch memory).
struct C4 {
  int x, y, z, t;
};
TM_HD int wrapc(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }
TM_HD C4 cc_coords(const CoarseGeom& g, long s) {
  C4 c;
  long r = s;
  c.x = (int)(r % g.L[0]); r /= g.L[0];
  c.y = (int)(r % g.L[1]); r /= g.L[1];
  c.z = (int)(r % g.L[2]);
  c.t = (int)(r / g.L[2]);
  return c;
}
TM_HD long cc_index(const CoarseGeom& g, C4 c) {
  return ((long)(c.t * g.L[2] + c.z) * g.L[1] + c.y) * g.L[0] + c.x;
}
TM_HD C4 cc_shift(const CoarseGeom& g, C4 c, int mu, int step) {
  C4 o = c;
  o.x = mu == 0 ? wrapc(c.x + step, g.L[0]) : c.x;
  o.y = mu == 1 ? wrapc(c.y + step, g.L[1]) : c.y;
  o.z = mu == 2 ? wrapc(c.z + step, g.L[2]) : c.z;
  o.t = mu == 3 ? wrapc(c.t + step, g.L[3]) : c.t;
  return o;
}
TM_HD long cc_nbr(const CoarseGeom& g, C4 c, int mu, int step) { return cc_index(g, cc_shift(g, c, mu, step)); }
TM_HD int c4_get(C4 c, int mu) { return mu == 0 ? c.x : (mu == 1 ? c.y : (mu == 2 ? c.z : c.t)); }
TM_HD int i4_get(const int* a, int mu) { return mu == 0 ? a[0] : (mu == 1 ? a[1] : (mu == 2 ? a[2] : a[3])); }

// ------------------------------------------------------------------ reductions
template <typename T> TM_D T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
