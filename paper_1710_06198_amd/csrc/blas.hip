// BLAS-1 with deterministic two-stage reductions (fixed block count, fixed
// summation order) and the small dense work of (F)GMRES on the device:
// Hessenberg columns, Givens rotations, per-RHS convergence flags and the
// final triangular solve.  Nothing here synchronises with the host, so a
// Krylov cycle can run as a fixed, predicated schedule of launches.
#include "kernels.h"

#include <algorithm>
#include <cmath>

static constexpr int RB = 256;   // threads per reduction block

int reduce_blocks(long n) {
  long nb = (n + RB * 8 - 1) / (RB * 8);
  return (int)std::max(1L, std::min(1024L, nb));
}

template <typename T> TM_D void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { red[2 * w] = a; red[2 * w + 1] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0; b = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { a += red[2 * i]; b += red[2 * i + 1]; }
  }
  __syncthreads();
}

// partial[(r*nvec + i)*NB + b] = sum over block b's chunk of conj(V_i,r) w_r;
// grid (NB, nvec, nrhs): every (chunk, vector) pair reduces in parallel.
template <typename T>
__global__ void __launch_bounds__(RB) k_multidot(const cplx<T>* __restrict__ V, long vstride, int nvec,
                                                 const cplx<T>* __restrict__ w, long n, double* partial, int NB,
                                                 const int* __restrict__ active) {
  __shared__ double red[2 * (RB / 64)];
  const int b = blockIdx.x, i = blockIdx.y, r = blockIdx.z;
  if (active && !active[r]) return;
  const long chunk = (n + NB - 1) / NB;
  const long lo = b * chunk, hi = min(n, lo + chunk);
  const cplx<T>* wr = w + (long)r * n;
  const cplx<T>* v = V + (long)i * vstride + (long)r * n;
  double are = 0, aim = 0;
  for (long k = lo + threadIdx.x; k < hi; k += RB) {
    cplx<T> a = v[k], c = wr[k];
    are += (double)a.re * c.re + (double)a.im * c.im;
    aim += (double)a.re * c.im - (double)a.im * c.re;
  }
  block_sum2<T>(are, aim, red);
  if (threadIdx.x == 0) {
    long o = ((long)r * nvec + i) * NB + b;
    partial[2 * o] = are;
    partial[2 * o + 1] = aim;
  }
}

template <typename T>
void launch_multidot(const cplx<T>* V, long vstride, int nvec, const cplx<T>* w, long n, int nrhs, double* partial,
                     int NB, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_multidot<T>, dim3(NB, nvec, nrhs), dim3(RB), 0, st, V, vstride, nvec, w, n, partial, NB,
                     active);
}

// out[(o / nvec)*ostride + o % nvec] = sum_b partial[o*NB + b] (complex), one wave per output
__global__ void k_finalize(const double* __restrict__ partial, int nout, int nvec, int NB, double* out, int ostride,
                           const int* __restrict__ mask) {
  const int o = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= nout) return;
  if (mask && !mask[o / nvec]) return;
  double a = 0, c = 0;
  for (int b = lane; b < NB; b += 64) { a += partial[2 * ((long)o * NB + b)]; c += partial[2 * ((long)o * NB + b) + 1]; }
  a = wave_sum(a);
  c = wave_sum(c);
  if (lane == 0) {
    long d = (long)(o / nvec) * ostride + (o % nvec);
    out[2 * d] = a;
    out[2 * d + 1] = c;
  }
}
void launch_finalize(const double* partial, int nout, int nvec, int NB, double* out, int ostride, hipStream_t st,
                     const int* mask) {
  hipLaunchKernelGGL(k_finalize, dim3((nout + 3) / 4), dim3(256), 0, st, partial, nout, nvec, NB, out, ostride, mask);
}

template <typename T>
__global__ void __launch_bounds__(RB) k_norm2(const cplx<T>* __restrict__ w, long n, double* partial, int NB,
                                              const int* __restrict__ active) {
  __shared__ double red[2 * (RB / 64)];
  const int r = blockIdx.y, b = blockIdx.x;
  if (active && !active[r]) return;
  const long chunk = (n + NB - 1) / NB;
  const long lo = b * chunk, hi = min(n, lo + chunk);
  const cplx<T>* wr = w + (long)r * n;
  double a = 0, z = 0;
  for (long k = lo + threadIdx.x; k < hi; k += RB) {
    cplx<T> v = wr[k];
    a += (double)v.re * v.re + (double)v.im * v.im;
  }
  block_sum2<T>(a, z, red);
  if (threadIdx.x == 0) partial[(long)r * NB + b] = a;
}
template <typename T>
void launch_norm2(const cplx<T>* w, long n, int nrhs, double* partial, int NB, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2<T>, dim3(NB, nrhs), dim3(RB), 0, st, w, n, partial, NB, active);
}
__global__ void k_finalize_real(const double* __restrict__ partial, int nout, int NB, double* out) {
  const int o = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (o >= nout) return;
  double a = 0;
  for (int b = lane; b < NB; b += 64) a += partial[(long)o * NB + b];
  a = wave_sum(a);
  if (lane == 0) out[o] = a;
}
void launch_finalize_real(const double* partial, int nout, int NB, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_real, dim3((nout + 3) / 4), dim3(256), 0, st, partial, nout, NB, out);
}

template <typename T>
__global__ void k_multiaxpy(cplx<T>* __restrict__ w, const cplx<T>* __restrict__ V, long vstride, int nvec,
                            const double* __restrict__ coef, int cstride, long n, double sign,
                            const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* cr = coef + 2L * r * cstride;
  cplx<T> acc = w[(long)r * n + k];
  for (int i = 0; i < nvec; ++i) {
    cplx<T> c = mk<T>((T)(sign * cr[2 * i]), (T)(sign * cr[2 * i + 1]));
    cfma(acc, c, V[(long)i * vstride + (long)r * n + k]);
  }
  w[(long)r * n + k] = acc;
}
template <typename T>
void launch_multiaxpy(cplx<T>* w, const cplx<T>* V, long vstride, int nvec, const double* coef, int cstride, long n,
                      int nrhs, double sign, const int* active, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_multiaxpy<T>, grid, dim3(256), 0, st, w, V, vstride, nvec, coef, cstride, n, sign, active);
}

// y may be x (in place): no restrict on the two
template <typename T>
__global__ void k_scale_dev(const cplx<T>* x, cplx<T>* y, const double* __restrict__ s, long n,
                            const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  T f = (T)s[r];
  y[(long)r * n + k] = f * x[(long)r * n + k];
}
template <typename T>
void launch_scale_dev(const cplx<T>* x, cplx<T>* y, const double* s, long n, int nrhs, const int* active,
                      hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_scale_dev<T>, grid, dim3(256), 0, st, x, y, s, n, active);
}

template <typename Tin, typename Tout>
__global__ void k_convert(const cplx<Tin>* __restrict__ x, cplx<Tout>* __restrict__ y, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x) {
    cplx<Tin> v = x[k];
    y[k] = mk<Tout>((Tout)v.re, (Tout)v.im);
  }
}
template <typename Tin, typename Tout>
void launch_convert(const cplx<Tin>* x, cplx<Tout>* y, long count, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(grid1d(count)), dim3(256), 0, st, x, y, count);
}

template <typename T>
__global__ void k_axpby(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, double a, double b, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x)
    y[k] = (T)a * x[k] + (T)b * y[k];
}
template <typename T>
void launch_axpby(const cplx<T>* x, cplx<T>* y, double a, double b, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid1d(count)), dim3(256), 0, st, x, y, a, b, count);
}
template <typename T>
__global__ void k_xmy(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x)
    y[k] = x[k] - y[k];
}
template <typename T>
void launch_xmy(const cplx<T>* x, cplx<T>* y, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_xmy<T>, dim3(grid1d(count)), dim3(256), 0, st, x, y, count);
}
template <typename T>
__global__ void k_add_to64(const cplx<T>* __restrict__ x, cplx<double>* __restrict__ y, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x) {
    cplx<T> v = x[k];
    y[k] += mk<double>((double)v.re, (double)v.im);
  }
}
template <typename T>
void launch_add_to64(const cplx<T>* x, cplx<double>* y, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_add_to64<T>, dim3(grid1d(count)), dim3(256), 0, st, x, y, count);
}

// Flavour coupling of the doublet operator (Sec. 1.1, Eq. 2): with the two
// flavours stored back to back (n elements each), y_f += a x_{1-f}.
template <typename T>
__global__ void k_flavour_couple(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, double a, long n) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < 2 * n; k += (long)gridDim.x * blockDim.x)
    y[k] += (T)a * x[k < n ? k + n : k - n];
}
template <typename T>
void launch_flavour_couple(const cplx<T>* x, cplx<T>* y, double a, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_flavour_couple<T>, dim3(grid1d(2 * n)), dim3(256), 0, st, x, y, a, n);
}

// out = a + c b for complex fields of n elements, c complex (host scalar)
__global__ void k_lincomb(const cplx<double>* __restrict__ a, const cplx<double>* __restrict__ b,
                          cplx<double>* __restrict__ out, double cre, double cim, long n) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    cplx<double> v = a[k];
    cfma(v, mk(cre, cim), b[k]);
    out[k] = v;
  }
}
void launch_lincomb(const cplx<double>* a, const cplx<double>* b, cplx<double>* out, double cre, double cim, long n,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(grid1d(n)), dim3(256), 0, st, a, b, out, cre, cim, n);
}

// plain streaming copy (one 16-byte access per thread); the reference
// kernel of known traffic for counter calibration and the measured copy
// ceiling (one element per thread beat grid-stride loops with 2048-65536
// workgroups and non-temporal variants on MI355X: 6.1 against 4.4-5.1 TB/s)
__global__ void k_copy16(const uint4* __restrict__ in, uint4* __restrict__ out, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}
void launch_copy16(const void* in, void* out, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const uint4*)in, (uint4*)out, n);
}

// 4-byte words; buffers of any size (the grid strides)
__global__ void k_fill_zero(uint32_t* p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0u;
}
void launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n = bytes / 4;
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid1d(n)), dim3(256), 0, st, (uint32_t*)p, n);
}

// ------------------------------------------------------------------ Krylov scalars
TM_D bool finite(double v) { return !(isnan(v) || isinf(v)); }

__global__ void k_krylov_start(KrylovDev k, double reltol, const double* abstol, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int m = k.m;
  double beta = sqrt(k.nrm[r]);
  k.beta0[r] = beta;
  double* g = k.g + 2L * r * (m + 1);
  for (int i = 0; i <= m; ++i) { g[2 * i] = 0; g[2 * i + 1] = 0; }
  g[0] = beta;
  double target = abstol ? abstol[r] : reltol * beta;
  k.tol[r] = target;
  k.kdone[r] = 0;
  k.inv[r] = beta > 0 ? 1.0 / beta : 0.0;
  if (!finite(beta)) { k.active[r] = 0; k.status[r] = 2; k.inv[r] = 0; }
  else if (beta <= target || beta == 0.0) { k.active[r] = 0; k.status[r] = 1; }
  else { k.active[r] = 1; k.status[r] = 0; }
}
void launch_krylov_start(const KrylovDev& k, double reltol, const double* abstol, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_krylov_start, dim3((nrhs + 63) / 64), dim3(64), 0, st, k, reltol, abstol, nrhs);
}

__global__ void k_cgs_decide(KrylovDev k, int j, int nrhs, double eta2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int m = k.m;
  const double* c1 = k.c1 + 2L * r * (m + 1);
  double* c2 = k.c2 + 2L * r * (m + 1);
  int need = 0;
  if (k.active[r]) {
    double s = 0;
    for (int i = 0; i <= j; ++i) s += c1[2 * i] * c1[2 * i] + c1[2 * i + 1] * c1[2 * i + 1];
    const double w2 = c1[2 * (j + 1)];
    need = !(w2 - s >= eta2 * w2);   // NaN takes the second pass too
  }
  k.reorth[r] = need;
  if (!need)
    for (int i = 0; i <= j; ++i) { c2[2 * i] = 0; c2[2 * i + 1] = 0; }
}
void launch_cgs_decide(const KrylovDev& k, int j, int nrhs, double eta2, hipStream_t st) {
  hipLaunchKernelGGL(k_cgs_decide, dim3((nrhs + 63) / 64), dim3(64), 0, st, k, j, nrhs, eta2);
}

__global__ void k_krylov_step(KrylovDev k, int j, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !k.active[r]) return;
  const int m = k.m;
  double* H = k.H + 2L * r * (m + 1) * m;     // H[i][j] at (i*m + j); column j built in place
  double* cs = k.cs + 2L * r * m;
  double* sn = k.sn + 2L * r * m;
  double* g = k.g + 2L * r * (m + 1);
  const double* c1 = k.c1 + 2L * r * (m + 1);
  const double* c2 = k.c2 + 2L * r * (m + 1);
  double hn = sqrt(fmax(k.nrm[r], 0.0));
  // column j = c1 + c2 with the previous rotations [[c, s], [-conj(s), conj(c)]] applied
  double ar = c1[0] + c2[0], ai = c1[1] + c2[1];
  for (int i = 0; i < j; ++i) {
    double br = c1[2 * (i + 1)] + c2[2 * (i + 1)], bi = c1[2 * (i + 1) + 1] + c2[2 * (i + 1) + 1];
    double cr = cs[2 * i], ci = cs[2 * i + 1], sr = sn[2 * i], si = sn[2 * i + 1];
    double tr = cr * ar - ci * ai + sr * br - si * bi;
    double ti = cr * ai + ci * ar + sr * bi + si * br;
    double ur = -(sr * ar + si * ai) + (cr * br + ci * bi);
    double ui = -(sr * ai - si * ar) + (cr * bi - ci * br);
    H[2 * (i * m + j)] = tr;
    H[2 * (i * m + j) + 1] = ti;
    ar = ur;
    ai = ui;
  }
  double den = sqrt(ar * ar + ai * ai + hn * hn);
  bool bad = !finite(den) || !finite(hn) || den == 0.0;
  if (bad) { k.active[r] = 0; k.status[r] = 2; k.inv[r] = 0; return; }
  // c = conj(a)/den, s = conj(b)/den with b = hn real
  cs[2 * j] = ar / den; cs[2 * j + 1] = -ai / den;
  sn[2 * j] = hn / den; sn[2 * j + 1] = 0;
  H[2 * (j * m + j)] = den;
  H[2 * (j * m + j) + 1] = 0;
  double gr = g[2 * j], gi = g[2 * j + 1];
  double s_r = hn / den;
  g[2 * (j + 1)] = -s_r * gr;
  g[2 * (j + 1) + 1] = -s_r * gi;
  double c_r = ar / den, c_i = -ai / den;
  g[2 * j] = c_r * gr - c_i * gi;
  g[2 * j + 1] = c_r * gi + c_i * gr;
  k.kdone[r] = j + 1;
  double res = sqrt(g[2 * (j + 1)] * g[2 * (j + 1)] + g[2 * (j + 1) + 1] * g[2 * (j + 1) + 1]);
  k.nrm[r] = res;      // implicit residual (for the host)
  if (hn <= 1e-300 || hn <= 1e-15 * den) {
    k.inv[r] = 0;
    k.active[r] = 0;
    k.status[r] = 1;   // invariant subspace: the solution is exact
  } else {
    k.inv[r] = 1.0 / hn;
    if (res <= k.tol[r]) { k.active[r] = 0; k.status[r] = 1; }
  }
  if (j + 1 >= m && k.active[r]) k.active[r] = 0;   // cycle exhausted; status stays 0
}
void launch_krylov_step(const KrylovDev& k, int j, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_krylov_step, dim3((nrhs + 63) / 64), dim3(64), 0, st, k, j, nrhs);
}

__global__ void k_krylov_solve_y(KrylovDev k, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int m = k.m;
  const int n = k.kdone[r];
  const double* H = k.H + 2L * r * (m + 1) * m;
  const double* g = k.g + 2L * r * (m + 1);
  double* y = k.y + 2L * r * m;
  for (int i = n - 1; i >= 0; --i) {
    double sr = g[2 * i], si = g[2 * i + 1];
    for (int l = i + 1; l < n; ++l) {
      double hr = H[2 * (i * m + l)], hi = H[2 * (i * m + l) + 1];
      sr -= hr * y[2 * l] - hi * y[2 * l + 1];
      si -= hr * y[2 * l + 1] + hi * y[2 * l];
    }
    double dr = H[2 * (i * m + i)], di = H[2 * (i * m + i) + 1];
    double dd = dr * dr + di * di;
    y[2 * i] = (sr * dr + si * di) / dd;
    y[2 * i + 1] = (si * dr - sr * di) / dd;
  }
}
void launch_krylov_solve_y(const KrylovDev& k, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_krylov_solve_y, dim3((nrhs + 63) / 64), dim3(64), 0, st, k, nrhs);
}

template <typename T>
__global__ void k_krylov_update(cplx<T>* __restrict__ x, const cplx<T>* __restrict__ Z, long zstride, KrylovDev k,
                                long n) {
  const int r = blockIdx.y;
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int nk = k.kdone[r];
  if (nk == 0) return;
  const double* y = k.y + 2L * r * k.m;
  cplx<T> acc = x[(long)r * n + e];
  for (int i = 0; i < nk; ++i) cfma(acc, mk<T>((T)y[2 * i], (T)y[2 * i + 1]), Z[(long)i * zstride + (long)r * n + e]);
  x[(long)r * n + e] = acc;
}
template <typename T>
void launch_krylov_update(cplx<T>* x, const cplx<T>* Z, long zstride, const KrylovDev& k, long n, int nrhs,
                          hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_krylov_update<T>, grid, dim3(256), 0, st, x, Z, zstride, k, n);
}

#define INST_T(T)                                                                                              \
  template void launch_multidot<T>(const cplx<T>*, long, int, const cplx<T>*, long, int, double*, int,         \
                                   const int*, hipStream_t);                                                   \
  template void launch_norm2<T>(const cplx<T>*, long, int, double*, int, const int*, hipStream_t);             \
  template void launch_multiaxpy<T>(cplx<T>*, const cplx<T>*, long, int, const double*, int, long, int, double, \
                                    const int*, hipStream_t);                                                  \
  template void launch_scale_dev<T>(const cplx<T>*, cplx<T>*, const double*, long, int, const int*,           \
                                    hipStream_t);                                                              \
  template void launch_axpby<T>(const cplx<T>*, cplx<T>*, double, double, long, hipStream_t);                  \
  template void launch_xmy<T>(const cplx<T>*, cplx<T>*, long, hipStream_t);                                    \
  template void launch_add_to64<T>(const cplx<T>*, cplx<double>*, long, hipStream_t);                          \
  template void launch_flavour_couple<T>(const cplx<T>*, cplx<T>*, double, long, hipStream_t);                 \
  template void launch_krylov_update<T>(cplx<T>*, const cplx<T>*, long, const KrylovDev&, long, int, hipStream_t);
INST_T(double)
INST_T(float)
template void launch_convert<double, float>(const cplx<double>*, cplx<float>*, long, hipStream_t);
template void launch_convert<float, double>(const cplx<float>*, cplx<double>*, long, hipStream_t);
template void launch_convert<double, double>(const cplx<double>*, cplx<double>*, long, hipStream_t);
template void launch_convert<float, float>(const cplx<float>*, cplx<float>*, long, hipStream_t);
