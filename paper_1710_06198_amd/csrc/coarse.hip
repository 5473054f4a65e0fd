// Coarse-level kernels: the coarse operator D_c(mu) = D_c + i mu Gamma5,c
// (Sec. 1.1), SAP on a coarse level, transfers between two coarse levels,
// block Gram-Schmidt of coarse test vectors, and the Galerkin product
// D_c' = P^dag D_c P for the next coarsening.
#include <type_traits>

#include "kernels.h"
#include "mfma.h"
#include "solver.h"

template <typename S> using SP = typename Store<S>::pair;

// ------------------------------------------------------------------ apply (K6)
// One thread per (site, row); the 9 input vectors a site needs are staged in LDS.
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_coarse_apply(CoarseGeom g, int d, const SP<S>* __restrict__ Dc,
                                                      const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                      const double* __restrict__ mu_dev) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int spw = 256 / d;
  const int ls = threadIdx.x / d, i = threadIdx.x - ls * d;
  const long y = (long)blockIdx.x * spw + ls;
  const int r = blockIdx.y;
  const bool valid = ls < spw && y < g.V;
  const cplx<T>* inr = in + (long)r * g.V * d;
  cplx<T>* st = lds + ls * 9 * d;
  if (valid) {
    const C4 c = cc_coords(g, y);
    st[i] = inr[y * d + i];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      st[(1 + 2 * mu) * d + i] = inr[cc_nbr(g, c, mu, +1) * d + i];
      st[(2 + 2 * mu) * d + i] = inr[cc_nbr(g, c, mu, -1) * d + i];
    }
  }
  __syncthreads();
  if (!valid) return;
  const SP<S>* D = Dc + y * 9L * d * d;
  cplx<T> acc = mk<T>(0, 0);
  for (int b = 0; b < 9; ++b) {
    const SP<S>* Db = D + (long)b * d * d + i;
    const cplx<T>* v = st + b * d;
    for (int j = 0; j < d; ++j) cfma(acc, Store<S>::template ld<T>(Db + (long)j * d), v[j]);
  }
  const T mu = (T)mu_dev[r];
  const T sg = i < d / 2 ? mu : -mu;
  acc += sg * times_i(st[i]);
  out[(long)r * g.V * d + y * d + i] = acc;
}

template <typename T, typename S, int D>
__global__ void __launch_bounds__(256) k_coarse_apply_d(CoarseGeom g, const SP<S>* __restrict__ Dc,
                                                        const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                        const double* __restrict__ mu_dev) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  constexpr int spw = 256 / D;
  const int ls = threadIdx.x / D, i = threadIdx.x - ls * D;
  const long y = (long)blockIdx.x * spw + ls;
  const int r = blockIdx.y;
  const bool valid = ls < spw && y < g.V;
  const cplx<T>* inr = in + (long)r * g.V * D;
  cplx<T>* st = lds + ls * 9 * D;
  if (valid) {
    const C4 c = cc_coords(g, y);
    st[i] = inr[y * D + i];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      st[(1 + 2 * mu) * D + i] = inr[cc_nbr(g, c, mu, +1) * D + i];
      st[(2 + 2 * mu) * D + i] = inr[cc_nbr(g, c, mu, -1) * D + i];
    }
  }
  __syncthreads();
  if (!valid) return;
  const SP<S>* Dm = Dc + y * 9L * D * D + i;
  cplx<T> acc = mk<T>(0, 0);
  for (int b = 0; b < 9; ++b) {
    const SP<S>* Db = Dm + (long)b * D * D;
    const cplx<T>* v = st + b * D;
#pragma unroll 16
    for (int j = 0; j < D; ++j) cfma(acc, Store<S>::template ld<T>(Db + j * D), v[j]);
  }
  const T mu = (T)mu_dev[r];
  acc += (i < D / 2 ? mu : -mu) * times_i(st[i]);
  out[(long)r * g.V * D + y * D + i] = acc;
}

template <typename T, typename S>
void launch_coarse_apply(const CoarseGeom& g, int d, const SP<S>* Dc, const cplx<T>* in, cplx<T>* out, int nrhs,
                         const double* mu_dev, hipStream_t st) {
  if (launch_coarse_apply_site<T, S>(g, d, Dc, in, out, nrhs, mu_dev, st)) return;
  const int spw = 256 / d;
  dim3 grid((unsigned)((g.V + spw - 1) / spw), nrhs);
  size_t sh = (size_t)spw * 9 * d * sizeof(cplx<T>);
  switch (d) {
    case 24: hipLaunchKernelGGL((k_coarse_apply_d<T, S, 24>), grid, dim3(256), sh, st, g, Dc, in, out, mu_dev); return;
    case 32: hipLaunchKernelGGL((k_coarse_apply_d<T, S, 32>), grid, dim3(256), sh, st, g, Dc, in, out, mu_dev); return;
    case 48: hipLaunchKernelGGL((k_coarse_apply_d<T, S, 48>), grid, dim3(256), sh, st, g, Dc, in, out, mu_dev); return;
    case 64: hipLaunchKernelGGL((k_coarse_apply_d<T, S, 64>), grid, dim3(256), sh, st, g, Dc, in, out, mu_dev); return;
    default: break;
  }
  hipLaunchKernelGGL((k_coarse_apply<T, S>), grid, dim3(256), sh, st, g, d, Dc, in, out, mu_dev);
}

template <typename T>
__global__ void k_gamma5_coarse(long n, int d, const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  int i = (int)(k % d);
  cplx<T> v = in[k];
  out[k] = i < d / 2 ? v : -v;
}
template <typename T>
void launch_gamma5_coarse(long V, int d, const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st) {
  long n = V * d * nrhs;
  hipLaunchKernelGGL(k_gamma5_coarse<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, d, in, out);
}

// ------------------------------------------------------------------ SAP on a coarse level
struct CBlock {
  int B[4], NB[4], nbs;
};
// site of local index sl in block blk: global coordinates c, local coordinates lc
TM_D void cblock_site(const CoarseGeom& g, const CBlock& cb, int blk, int sl, C4& c, C4& lc) {
  int b = blk;
  const int bc0 = b % cb.NB[0]; b /= cb.NB[0];
  const int bc1 = b % cb.NB[1]; b /= cb.NB[1];
  const int bc2 = b % cb.NB[2];
  const int bc3 = b / cb.NB[2];
  int l = sl;
  lc.x = l % cb.B[0]; l /= cb.B[0];
  lc.y = l % cb.B[1]; l /= cb.B[1];
  lc.z = l % cb.B[2];
  lc.t = l / cb.B[2];
  c.x = bc0 * cb.B[0] + lc.x;
  c.y = bc1 * cb.B[1] + lc.y;
  c.z = bc2 * cb.B[2] + lc.z;
  c.t = bc3 * cb.B[3] + lc.t;
}
// local index of the neighbour inside the block, or -1 when it lies outside
TM_D int cblock_nbr_local(const CBlock& cb, C4 lc, int mu, int step) {
  const int Bm = i4_get(cb.B, mu), NBm = i4_get(cb.NB, mu);
  int v = c4_get(lc, mu) + step;
  if (v < 0 || v >= Bm) {
    if (NBm != 1) return -1;
    v = v < 0 ? v + Bm : v - Bm;
  }
  C4 l2 = lc;
  l2.x = mu == 0 ? v : lc.x;
  l2.y = mu == 1 ? v : lc.y;
  l2.z = mu == 2 ? v : lc.z;
  l2.t = mu == 3 ? v : lc.t;
  return ((l2.t * cb.B[2] + l2.z) * cb.B[1] + l2.y) * cb.B[0] + l2.x;
}

template <typename T>
TM_D void block_reduce3c(T& a, T& b, T& c, T* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  if (lane == 0) { red[w * 3] = a; red[w * 3 + 1] = b; red[w * 3 + 2] = c; }
  __syncthreads();
  a = 0; b = 0; c = 0;
  for (int k = 0; k < nw; ++k) { a += red[k * 3]; b += red[k * 3 + 1]; c += red[k * 3 + 2]; }
  __syncthreads();
}

template <typename T, typename S, int EPT>
__global__ void __launch_bounds__(256) k_sap_coarse(CoarseGeom g, int d, CBlock cb, const SP<S>* __restrict__ Dc,
                                                    const cplx<T>* __restrict__ eta, cplx<T>* z,
                                                    const double* __restrict__ mu_dev, const int* __restrict__ blist,
                                                    int mr_steps) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nel = cb.nbs * d;
  T* red = reinterpret_cast<T*>(lds + nel);
  const int r = blockIdx.y;
  const int blk = blist[blockIdx.x];
  const T mu = (T)mu_dev[r];
  const cplx<T>* er = eta + (long)r * g.V * d;
  cplx<T>* zr = z + (long)r * g.V * d;
  cplx<T> rho[EPT], e[EPT], q[EPT];
  // residual r = eta - D_c z on the block
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    int el = threadIdx.x + k * 256;
    rho[k] = mk<T>(0, 0);
    e[k] = mk<T>(0, 0);
    if (el < nel) {
      int sl = el / d, i = el - sl * d;
      C4 c, lc;
      cblock_site(g, cb, blk, sl, c, lc);
      long y = cc_index(g, c);
      const SP<S>* D = Dc + y * 9L * d * d + i;
      cplx<T> acc = mk<T>(0, 0);
      for (int b = 0; b < 9; ++b) {
        long src = b == 0 ? y : cc_nbr(g, c, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
        const cplx<T>* v = zr + src * d;
        const SP<S>* Db = D + (long)b * d * d;
        for (int j = 0; j < d; ++j) cfma(acc, Store<S>::template ld<T>(Db + (long)j * d), v[j]);
      }
      cplx<T> zi = zr[y * d + i];
      acc += (i < d / 2 ? mu : -mu) * times_i(zi);
      rho[k] = er[y * d + i] - acc;
    }
  }
  for (int it = 0; it < mr_steps; ++it) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int el = threadIdx.x + k * 256;
      if (el < nel) lds[el] = rho[k];
    }
    __syncthreads();
    T qq = 0, qre = 0, qim = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int el = threadIdx.x + k * 256;
      q[k] = mk<T>(0, 0);
      if (el < nel) {
        int sl = el / d, i = el - sl * d;
        C4 c, lc;
        cblock_site(g, cb, blk, sl, c, lc);
        long y = cc_index(g, c);
        const SP<S>* D = Dc + y * 9L * d * d + i;
        cplx<T> acc = mk<T>(0, 0);
        for (int b = 0; b < 9; ++b) {
          int nl = b == 0 ? sl : cblock_nbr_local(cb, lc, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
          if (nl < 0) continue;
          const cplx<T>* v = lds + nl * d;
          const SP<S>* Db = D + (long)b * d * d;
          for (int j = 0; j < d; ++j) cfma(acc, Store<S>::template ld<T>(Db + (long)j * d), v[j]);
        }
        acc += (i < d / 2 ? mu : -mu) * times_i(rho[k]);
        q[k] = acc;
        qq += norm2(acc);
        cplx<T> t = cmulc(acc, rho[k]);
        qre += t.re;
        qim += t.im;
      }
    }
    block_reduce3c(qq, qre, qim, red);
    cplx<T> alpha = qq > (T)0 ? mk(qre / qq, qim / qq) : mk<T>(0, 0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      cfma(e[k], alpha, rho[k]);
      rho[k] -= alpha * q[k];
    }
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    int el = threadIdx.x + k * 256;
    if (el < nel) {
      int sl = el / d, i = el - sl * d;
      C4 c, lc;
      cblock_site(g, cb, blk, sl, c, lc);
      long y = cc_index(g, c);
      zr[y * d + i] += e[k];
    }
  }
}

// Same block solve with the dof count fixed at compile time: 512 threads,
// up to 8 rows per thread, inner products partially unrolled.  The block
// correction is added to z after every MR step (z of a block is read only
// when its residual is formed, before the first step).
template <typename T, typename S, int D>
__global__ void __launch_bounds__(512) k_sap_coarse_d(CoarseGeom g, CBlock cb, const SP<S>* __restrict__ Dc,
                                                      const cplx<T>* __restrict__ eta, cplx<T>* z,
                                                      const double* __restrict__ mu_dev, const int* __restrict__ blist,
                                                      int mr_steps) {
  constexpr int EPT = 8;
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nel = cb.nbs * D;
  T* red = reinterpret_cast<T*>(lds + nel);
  const int r = blockIdx.y;
  const int blk = blist[blockIdx.x];
  const T mu = (T)mu_dev[r];
  const cplx<T>* er = eta + (long)r * g.V * D;
  cplx<T>* zr = z + (long)r * g.V * D;
  cplx<T> rho[EPT], q[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int el = threadIdx.x + k * 512;
    rho[k] = mk<T>(0, 0);
    if (el < nel) {
      const int sl = el / D, i = el - sl * D;
      C4 c, lc;
      cblock_site(g, cb, blk, sl, c, lc);
      const long y = cc_index(g, c);
      const SP<S>* Dm = Dc + y * 9L * D * D + i;
      cplx<T> acc = mk<T>(0, 0);
      for (int b = 0; b < 9; ++b) {
        long src = b == 0 ? y : cc_nbr(g, c, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
        const cplx<T>* v = zr + src * D;
        const SP<S>* Db = Dm + (long)b * D * D;
#pragma unroll 8
        for (int j = 0; j < D; ++j) cfma(acc, Store<S>::template ld<T>(Db + j * D), v[j]);
      }
      acc += (i < D / 2 ? mu : -mu) * times_i(zr[y * D + i]);
      rho[k] = er[y * D + i] - acc;
    }
  }
  __syncthreads();   // every residual is formed before z changes
  for (int it = 0; it < mr_steps; ++it) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int el = threadIdx.x + k * 512;
      if (el < nel) lds[el] = rho[k];
    }
    __syncthreads();
    T qq = 0, qre = 0, qim = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int el = threadIdx.x + k * 512;
      q[k] = mk<T>(0, 0);
      if (el < nel) {
        const int sl = el / D, i = el - sl * D;
        C4 c, lc;
        cblock_site(g, cb, blk, sl, c, lc);
        const long y = cc_index(g, c);
        const SP<S>* Dm = Dc + y * 9L * D * D + i;
        cplx<T> acc = mk<T>(0, 0);
        for (int b = 0; b < 9; ++b) {
          const int nl = b == 0 ? sl : cblock_nbr_local(cb, lc, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
          if (nl < 0) continue;
          const cplx<T>* v = lds + nl * D;
          const SP<S>* Db = Dm + (long)b * D * D;
#pragma unroll 8
          for (int j = 0; j < D; ++j) cfma(acc, Store<S>::template ld<T>(Db + j * D), v[j]);
        }
        acc += (i < D / 2 ? mu : -mu) * times_i(rho[k]);
        q[k] = acc;
        qq += norm2(acc);
        cplx<T> t = cmulc(acc, rho[k]);
        qre += t.re;
        qim += t.im;
      }
    }
    block_reduce3c(qq, qre, qim, red);
    const cplx<T> alpha = qq > (T)0 ? mk(qre / qq, qim / qq) : mk<T>(0, 0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int el = threadIdx.x + k * 512;
      if (el < nel) {
        const int sl = el / D, i = el - sl * D;
        C4 c, lc;
        cblock_site(g, cb, blk, sl, c, lc);
        const long y = cc_index(g, c);
        cfma(zr[y * D + i], alpha, rho[k]);
      }
      rho[k] -= alpha * q[k];
    }
  }
}

template <typename T, typename S>
void launch_sap_coarse(const CoarseGeom& g, int d, const int blk[4], const SP<S>* Dc, const cplx<T>* eta, cplx<T>* z,
                       int nrhs, const double* mu_dev, const int* blist, int nblk, int mr_steps, hipStream_t st) {
  CBlock cb;
  cb.nbs = 1;
  for (int m = 0; m < 4; ++m) { cb.B[m] = blk[m]; cb.NB[m] = g.L[m] / blk[m]; cb.nbs *= blk[m]; }
  int nel = cb.nbs * d;
  size_t sh = (size_t)nel * sizeof(cplx<T>) + 3 * 4 * sizeof(T);
  dim3 grid(nblk, nrhs);
  if (nel <= 8 * 512 && (d == 24 || d == 32 || d == 48 || d == 64)) {
    size_t sh2 = (size_t)nel * sizeof(cplx<T>) + 3 * 16 * sizeof(T);
    if (d == 24)
      hipLaunchKernelGGL((k_sap_coarse_d<T, S, 24>), grid, dim3(512), sh2, st, g, cb, Dc, eta, z, mu_dev, blist, mr_steps);
    else if (d == 32)
      hipLaunchKernelGGL((k_sap_coarse_d<T, S, 32>), grid, dim3(512), sh2, st, g, cb, Dc, eta, z, mu_dev, blist, mr_steps);
    else if (d == 48)
      hipLaunchKernelGGL((k_sap_coarse_d<T, S, 48>), grid, dim3(512), sh2, st, g, cb, Dc, eta, z, mu_dev, blist, mr_steps);
    else
      hipLaunchKernelGGL((k_sap_coarse_d<T, S, 64>), grid, dim3(512), sh2, st, g, cb, Dc, eta, z, mu_dev, blist, mr_steps);
    return;
  }
  if (nel <= 4 * 256)
    hipLaunchKernelGGL((k_sap_coarse<T, S, 4>), grid, dim3(256), sh, st, g, d, cb, Dc, eta, z, mu_dev, blist,
                       mr_steps);
  else
    hipLaunchKernelGGL((k_sap_coarse<T, S, 16>), grid, dim3(256), sh, st, g, d, cb, Dc, eta, z, mu_dev, blist,
                       mr_steps);
}

// ------------------------------------------------------------------ transfers (K4/K5)
struct CAgg {
  int A[4], NA[4], na;   // aggregate extents, aggregates per dim, sites per aggregate
};
TM_HD CAgg make_cagg(const CoarseGeom& g, const int agg[4]) {
  CAgg a;
  a.na = 1;
  for (int m = 0; m < 4; ++m) { a.A[m] = agg[m]; a.NA[m] = g.L[m] / agg[m]; a.na *= agg[m]; }
  return a;
}
// global index of local site sl of aggregate Y (and its local coordinates)
TM_D long cagg_site(const CoarseGeom& g, const CAgg& a, long Y, int sl, int lc[4]) {
  long b = Y;
  int y0 = (int)(b % a.NA[0]); b /= a.NA[0];
  int y1 = (int)(b % a.NA[1]); b /= a.NA[1];
  int y2 = (int)(b % a.NA[2]);
  int y3 = (int)(b / a.NA[2]);
  int l = sl;
  lc[0] = l % a.A[0]; l /= a.A[0];
  lc[1] = l % a.A[1]; l /= a.A[1];
  lc[2] = l % a.A[2];
  lc[3] = l / a.A[2];
  int c[4] = {y0 * a.A[0] + lc[0], y1 * a.A[1] + lc[1], y2 * a.A[2] + lc[2], y3 * a.A[3] + lc[3]};
  return coarse_index(g, c);
}
TM_D long cagg_of(const CoarseGeom& g, const CAgg& a, const int c[4]) {
  return ((long)((c[3] / a.A[3]) * a.NA[2] + c[2] / a.A[2]) * a.NA[1] + c[1] / a.A[1]) * a.NA[0] + c[0] / a.A[0];
}

// out(Y, s*nv + i) = sum_{y in Y, k in half s} conj(P_i(y)_k) in(y)_k
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_restrict_coarse(CoarseGeom g, int d, CAgg a, const SP<S>* __restrict__ P,
                                                         int nv, const cplx<T>* __restrict__ in,
                                                         cplx<T>* __restrict__ out, long Vc) {
  __shared__ cplx<T> red[256];
  const long Y = blockIdx.x;
  const int r = blockIdx.y;
  const int no = 2 * nv;
  const int G = max(1, 256 / no);
  const int t = threadIdx.x, n = t % no, grp = t / no;
  const int hd = d / 2;
  cplx<T> acc = mk<T>(0, 0);
  if (grp < G) {
    const int s = n / nv, iv = n - s * nv;
    const SP<S>* Pi = P + (long)iv * g.V * d;
    const cplx<T>* inr = in + (long)r * g.V * d;
    for (int sl = grp; sl < a.na; sl += G) {
      int lc[4];
      long y = cagg_site(g, a, Y, sl, lc);
      for (int k = 0; k < hd; ++k) {
        long o = y * d + s * hd + k;
        cfmac(acc, Store<S>::template ld<T>(Pi + o), inr[o]);
      }
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < no) {
    cplx<T> sum = mk<T>(0, 0);
    for (int k = 0; k < G; ++k) sum += red[k * no + t];
    out[((long)r * Vc + Y) * no + t] = sum;
  }
}

// P^dag for 16 right-hand sides per workgroup on the matrix cores (FP32
// vectors, bf16 P, N_v <= 32, d/2 a multiple of 4): per coarse aggregate
// and chirality an (N_v x K) x (K x 16) product over K = sites x d/2,
// P exact in bf16, the inputs split into two bf16 parts (kept to 2^-18 of
// their size).  Wave w owns chirality w / 2 and vector tile w % 2; each lane
// group takes four consecutive components of one site per K step (one
// 16-byte load of P, two of the input).
__global__ void __launch_bounds__(256) k_restrict_coarse_mf(CoarseGeom g, int d, CAgg a,
                                                            const bf16pair* __restrict__ P, int nv,
                                                            const cplx<float>* __restrict__ in,
                                                            cplx<float>* __restrict__ out, long Vc, int nrhs) {
  __shared__ long sites[256];
  constexpr int NR = 16;
  const int ng = (nrhs + NR - 1) / NR;
  const int x8 = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int r0 = (rest % ng) * NR;
  const long Y = (long)(rest / ng) * 8 + x8;
  if (Y >= Vc) return;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  for (int sl = t; sl < a.na; sl += 256) {
    int lc[4];
    sites[sl] = cagg_site(g, a, Y, sl, lc);
  }
  __syncthreads();
  const int hd = d / 2, no = 2 * nv;
  const int sc = wv >> 1, mt = wv & 1, iv = 16 * mt + lr, r = r0 + lr;
  const unsigned* pbase = reinterpret_cast<const unsigned*>(P) + (long)(iv < nv ? iv : 0) * g.V * d + sc * hd;
  const cplx<float>* ibase = in + (long)(r < nrhs ? r : r0) * g.V * d + sc * hd;
  const int K = a.na * hd;
  mf_f4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kk = k0 + 4 * lk;   // four consecutive components of one site (hd % 4 == 0)
    uint4 pu = make_uint4(0u, 0u, 0u, 0u);
    float4 z01 = make_float4(0.f, 0.f, 0.f, 0.f), z23 = z01;
    if (kk < K) {
      const int sl = kk / hd, k = kk - sl * hd;
      const long o = sites[sl] * d + k;
      if (iv < nv) pu = *reinterpret_cast<const uint4*>(pbase + o);
      if (r < nrhs) {
        z01 = reinterpret_cast<const float4*>(ibase + o)[0];
        z23 = reinterpret_cast<const float4*>(ibase + o)[1];
      }
    }
    const unsigned pw[4] = {pu.x, pu.y, pu.z, pu.w};
    mf_s4 ar, ai;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ar[e] = (short)(pw[e] & 0xffffu);
      ai[e] = (short)(pw[e] >> 16);
    }
    const cplx<float> zv[4] = {mk(z01.x, z01.y), mk(z01.z, z01.w), mk(z23.x, z23.y), mk(z23.z, z23.w)};
    const MfSplit bb = mf_split(zv);
    mf_cmac_conj(ar, ai, bb, accr, acci);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int ivo = 16 * mt + 4 * lk + v, rr = r0 + lr;
    if (ivo < nv && rr < nrhs) out[((long)rr * Vc + Y) * no + sc * nv + ivo] = mk(accr[v], acci[v]);
  }
}

template <typename T, typename S>
void launch_restrict_coarse(const CoarseGeom& g, int d, const int agg[4], const SP<S>* P, int nv, const cplx<T>* in,
                            cplx<T>* out, int nrhs, hipStream_t st) {
  CAgg a = make_cagg(g, agg);
  long Vc = g.V / a.na;
  if constexpr (std::is_same<T, float>::value && std::is_same<S, __hip_bfloat16>::value) {
    if (nrhs >= 8 && nv <= 32 && (d / 2) % 4 == 0 && a.na <= 256) {
      const long n8 = (Vc + 7) / 8 * 8;
      hipLaunchKernelGGL(k_restrict_coarse_mf, dim3((unsigned)(n8 * ((nrhs + 15) / 16))), dim3(256), 0, st, g, d, a, P,
                         nv, in, out, Vc, nrhs);
      return;
    }
  }
  hipLaunchKernelGGL((k_restrict_coarse<T, S>), dim3((unsigned)Vc, nrhs), dim3(256), 0, st, g, d, a, P, nv, in, out,
                     Vc);
}

// out(y)_k = sum_i P_i(y)_k in(Y(y), s(k)*nv + i)
template <typename T, typename S>
__global__ void k_prolong_coarse(CoarseGeom g, int d, CAgg a, const SP<S>* __restrict__ P, int nv,
                                 const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, long Vc) {
  long el = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (el >= g.V * d) return;
  long y = el / d;
  int k = (int)(el - y * d);
  int c[4];
  coarse_coords(g, y, c);
  long Y = cagg_of(g, a, c);
  const int s = k < d / 2 ? 0 : 1;
  const cplx<T>* e = in + ((long)r * Vc + Y) * 2 * nv + s * nv;
  cplx<T> acc = mk<T>(0, 0);
  for (int i = 0; i < nv; ++i) cfma(acc, Store<S>::template ld<T>(P + (long)i * g.V * d + el), e[i]);
  out[(long)r * g.V * d + el] = acc;
}
template <typename T, typename S>
void launch_prolong_coarse(const CoarseGeom& g, int d, const int agg[4], const SP<S>* P, int nv, const cplx<T>* in,
                           cplx<T>* out, int nrhs, hipStream_t st) {
  CAgg a = make_cagg(g, agg);
  long Vc = g.V / a.na;
  long n = g.V * d;
  hipLaunchKernelGGL((k_prolong_coarse<T, S>), dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, g, d, a, P,
                     nv, in, out, Vc);
}

// ------------------------------------------------------------------ block Gram-Schmidt (K7)
// One workgroup per (aggregate, chirality): CGS with one re-orthogonalisation
// pass in FP64, vectors in index order; the pieces are kept in P64.
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_gs_coarse(CoarseGeom g, int d, CAgg a, const cplx<T>* __restrict__ tv,
                                                   int nv, cplx<double>* P64, SP<S>* P) {
  __shared__ double red[4][2 * 64];
  const long Y = blockIdx.x;
  const int s = blockIdx.y;
  const int hd = d / 2;
  const int nel = a.na * hd;
  constexpr int EPT = 4;
  long off[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    int el = threadIdx.x + k * 256;
    off[k] = -1;
    if (el < nel) {
      int sl = el / hd, kk = el - sl * hd;
      int lc[4];
      long y = cagg_site(g, a, Y, sl, lc);
      off[k] = y * d + s * hd + kk;
    }
  }
  const long vs = g.V * d;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < nv; ++i) {
    cplx<double> x[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      x[k] = mk(0.0, 0.0);
      if (off[k] >= 0) { cplx<T> v = tv[(long)i * vs + off[k]]; x[k] = mk((double)v.re, (double)v.im); }
    }
    for (int pass = 0; pass < 2 && i > 0; ++pass) {
      for (int j0 = 0; j0 < i; j0 += 64) {
        int nj = min(64, i - j0);
        for (int jj = 0; jj < nj; ++jj) {
          cplx<double> p = mk(0.0, 0.0);
#pragma unroll
          for (int k = 0; k < EPT; ++k)
            if (off[k] >= 0) cfmac(p, P64[(long)(j0 + jj) * vs + off[k]], x[k]);
          p.re = wave_sum(p.re);
          p.im = wave_sum(p.im);
          if (lane == 0) { red[w][2 * jj] = p.re; red[w][2 * jj + 1] = p.im; }
        }
        __syncthreads();
        for (int jj = 0; jj < nj; ++jj) {
          cplx<double> cj = mk(0.0, 0.0);
          for (int ww = 0; ww < 4; ++ww) cj += mk(red[ww][2 * jj], red[ww][2 * jj + 1]);
#pragma unroll
          for (int k = 0; k < EPT; ++k)
            if (off[k] >= 0) x[k] -= cj * P64[(long)(j0 + jj) * vs + off[k]];
        }
        __syncthreads();
      }
    }
    double nn = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) nn += norm2(x[k]);
    nn = wave_sum(nn);
    if (lane == 0) red[w][0] = nn;
    __syncthreads();
    nn = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    __syncthreads();
    double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (off[k] >= 0) {
        cplx<double> q = inv * x[k];
        P64[(long)i * vs + off[k]] = q;
        Store<S>::st(P + (long)i * vs + off[k], q);
      }
  }
}
template <typename T, typename S>
void launch_gs_coarse(const CoarseGeom& g, int d, const int agg[4], const cplx<T>* tv, int nv, cplx<double>* P64,
                      SP<S>* P, hipStream_t st) {
  CAgg a = make_cagg(g, agg);
  long Vc = g.V / a.na;
  hipLaunchKernelGGL((k_gs_coarse<T, S>), dim3((unsigned)Vc, 2), dim3(256), 0, st, g, d, a, tv, nv, P64, P);
}

// ------------------------------------------------------------------ Galerkin (K8), coarse -> coarser
// Workgroup per (aggregate Y, coarse column cc = s'*nv + j).  w = column cc
// of P on Y.  Stage 1 pushes w through each part of D_c (aggregate-internal
// couplings, and the face-crossing hops into each neighbour aggregate) into
// LDS; stage 2 projects each part onto P of the receiving aggregate.
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_galerkin_coarse(CoarseGeom g, int d, CAgg a, const SP<S>* __restrict__ Dc1,
                                                         const SP<S>* __restrict__ P, int nv, SP<S>* Dc2,
                                                         CoarseGeom g2) {
  extern __shared__ unsigned char smem_raw[];
  const int na = a.na;
  const int nel = na * d;
  cplx<T>* w = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* u = w + nel;
  long* tgt = reinterpret_cast<long*>(u + nel);
  cplx<T>* red = reinterpret_cast<cplx<T>*>(tgt + na);
  const long Y = blockIdx.x;
  const int cc = blockIdx.y;
  const int sp = cc / nv, jv = cc - sp * nv;
  const int hd = d / 2;
  const long vs = g.V * d;
  const int d2 = 2 * nv;
  // load w
  for (int el = threadIdx.x; el < nel; el += 256) {
    int sl = el / d, k = el - sl * d;
    int lc[4];
    long y = cagg_site(g, a, Y, sl, lc);
    bool in_s = (k < hd) == (sp == 0);
    w[el] = in_s ? Store<S>::template ld<T>(P + (long)jv * vs + y * d + k) : mk<T>(0, 0);
  }
  __syncthreads();
  for (int part = 0; part < 9; ++part) {
    // part 0: self; part 1+2mu: forward hops landing in Y - mu; part 2+2mu: backward hops landing in Y + mu
    const int mu = (part - 1) >> 1;
    const int step = ((part - 1) & 1) ? -1 : 1;
    for (int el = threadIdx.x; el < nel; el += 256) {
      int sl = el / d, i = el - sl * d;
      int lc[4];
      long y = cagg_site(g, a, Y, sl, lc);
      int c[4];
      coarse_coords(g, y, c);
      cplx<T> acc = mk<T>(0, 0);
      if (part == 0) {
        if (i == 0) tgt[sl] = y;
        const SP<S>* D = Dc1 + y * 9L * d * d + i;
        for (int b = 0; b < 9; ++b) {
          int nl;
          if (b == 0) nl = sl;
          else {
            int m = (b - 1) >> 1, stp = ((b - 1) & 1) ? -1 : 1;
            int v = lc[m] + stp;
            if (v < 0 || v >= a.A[m]) continue;   // face-crossing: not part of the self block
            int l2[4] = {lc[0], lc[1], lc[2], lc[3]};
            l2[m] = v;
            nl = ((l2[3] * a.A[2] + l2[2]) * a.A[1] + l2[1]) * a.A[0] + l2[0];
          }
          const SP<S>* Db = D + (long)b * d * d;
          const cplx<T>* v = w + nl * d;
          for (int j = 0; j < d; ++j) cfma(acc, Store<S>::template ld<T>(Db + (long)j * d), v[j]);
        }
      } else {
        // forward part: sources on the lower face of Y feed target t = y - mu through block 1+2mu of t;
        // backward part: sources on the upper face feed t = y + mu through block 2+2mu of t.
        bool face = step > 0 ? (lc[mu] == 0) : (lc[mu] == a.A[mu] - 1);
        if (face) {
          long t = coarse_neighbour(g, c, mu, -step);
          if (i == 0) tgt[sl] = t;
          const SP<S>* Db = Dc1 + t * 9L * d * d + (long)part * d * d + i;
          const cplx<T>* v = w + sl * d;
          for (int j = 0; j < d; ++j) cfma(acc, Store<S>::template ld<T>(Db + (long)j * d), v[j]);
        } else if (i == 0) {
          tgt[sl] = -1;
        }
      }
      u[el] = acc;
    }
    __syncthreads();
    // stage 2: project onto P of the receiving aggregate
    const int G = max(1, 256 / d2);
    const int t = threadIdx.x, n = t % d2, grp = t / d2;
    cplx<T> acc = mk<T>(0, 0);
    long recv = -1;
    if (grp < G) {
      const int s = n / nv, iv = n - s * nv;
      for (int sl = grp; sl < na; sl += G) {
        long ts = tgt[sl];
        if (ts < 0) continue;
        const SP<S>* Pi = P + (long)iv * vs + ts * d + s * hd;
        const cplx<T>* uu = u + sl * d + s * hd;
        for (int k = 0; k < hd; ++k) cfmac(acc, Store<S>::template ld<T>(Pi + k), uu[k]);
      }
    }
    red[t] = acc;
    __syncthreads();
    if (t < d2) {
      cplx<T> sum = mk<T>(0, 0);
      for (int k = 0; k < G; ++k) sum += red[k * d2 + t];
      // receiving aggregate
      if (part == 0) recv = Y;
      else {
        int yc[4];
        long b = Y;
        yc[0] = (int)(b % a.NA[0]); b /= a.NA[0];
        yc[1] = (int)(b % a.NA[1]); b /= a.NA[1];
        yc[2] = (int)(b % a.NA[2]);
        yc[3] = (int)(b / a.NA[2]);
        recv = coarse_neighbour(g2, yc, mu, -step);
      }
      Store<S>::st(Dc2 + ((recv * 9 + part) * (long)d2 + cc) * d2 + t, sum);
    }
    __syncthreads();
  }
}

// The same product with GC columns per workgroup: workgroup (Y, s', group)
// takes the columns cc = s' nv + g GC + c, c < GC, which all live on the
// s' half of the aggregate's components.  Each D_c element loaded in stage
// 1 serves the GC columns (w in LDS, [site][half component][column]);
// stage 2 gives each thread one output row n for GC / 4 columns.
constexpr int GAL_GC = 8;

template <typename T, typename S>
__global__ void __launch_bounds__(256) k_galerkin_coarse_cols(CoarseGeom g, int d, CAgg a,
                                                              const SP<S>* __restrict__ Dc1,
                                                              const SP<S>* __restrict__ P, int nv,
                                                              SP<S>* __restrict__ Dc2, CoarseGeom g2) {
  constexpr int GC = GAL_GC, CPT = GC / 4;   // columns per thread in stage 2 (one wave per CPT columns)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int na = a.na, hd = d / 2, d2 = 2 * nv;
  cplx<T>* w = reinterpret_cast<cplx<T>*>(smem_raw);   // [na][hd][GC]
  cplx<T>* u = w + (size_t)na * hd * GC;                // [na][d][GC]
  long* tgt = reinterpret_cast<long*>(u + (size_t)na * d * GC);
  const long Y = blockIdx.x;
  const int sp = blockIdx.y, jv0 = blockIdx.z * GC;
  const long vs = g.V * d;
  const int t = threadIdx.x;
  for (int e = t; e < na * hd * GC; e += 256) {
    const int c = e % GC, rem = e / GC, k = rem % hd, sl = rem / hd;
    int lc[4];
    const long y = cagg_site(g, a, Y, sl, lc);
    w[e] = jv0 + c < nv ? Store<S>::template ld<T>(P + (long)(jv0 + c) * vs + y * d + sp * hd + k) : mk<T>(0, 0);
  }
  __syncthreads();
  for (int part = 0; part < 9; ++part) {
    const int mu = (part - 1) >> 1;
    const int step = ((part - 1) & 1) ? -1 : 1;
    // stage 1: u = (part of D_c) w, rows (sl, i) over threads
    for (int row = t; row < na * d; row += 256) {
      const int sl = row / d, i = row - sl * d;
      int lc[4];
      const long y = cagg_site(g, a, Y, sl, lc);
      int c[4];
      coarse_coords(g, y, c);
      cplx<T> acc[GC];
#pragma unroll
      for (int q = 0; q < GC; ++q) acc[q] = mk<T>(0, 0);
      bool any = false;
      if (part == 0) {
        if (i == 0) tgt[sl] = y;
        any = true;
        for (int b = 0; b < 9; ++b) {
          int nl;
          if (b == 0) nl = sl;
          else {
            const int m = (b - 1) >> 1, stp = ((b - 1) & 1) ? -1 : 1;
            const int v = lc[m] + stp;
            if (v < 0 || v >= a.A[m]) continue;   // leaves the aggregate: a face part
            int l2[4] = {lc[0], lc[1], lc[2], lc[3]};
            l2[m] = v;
            nl = ((l2[3] * a.A[2] + l2[2]) * a.A[1] + l2[1]) * a.A[0] + l2[0];
          }
          const SP<S>* Db = Dc1 + (y * 9L + b) * d * d + (long)sp * hd * d + i;
          const cplx<T>* wn = w + (size_t)nl * hd * GC;
          for (int k = 0; k < hd; ++k) {
            const cplx<T> dv = Store<S>::template ld<T>(Db + (long)k * d);
#pragma unroll
            for (int q = 0; q < GC; ++q) cfma(acc[q], dv, wn[k * GC + q]);
          }
        }
      } else {
        const bool face = step > 0 ? (lc[mu] == 0) : (lc[mu] == a.A[mu] - 1);
        if (face) {
          const long tt = coarse_neighbour(g, c, mu, -step);
          if (i == 0) tgt[sl] = tt;
          any = true;
          const SP<S>* Db = Dc1 + (tt * 9L + part) * d * d + (long)sp * hd * d + i;
          const cplx<T>* wn = w + (size_t)sl * hd * GC;
          for (int k = 0; k < hd; ++k) {
            const cplx<T> dv = Store<S>::template ld<T>(Db + (long)k * d);
#pragma unroll
            for (int q = 0; q < GC; ++q) cfma(acc[q], dv, wn[k * GC + q]);
          }
        } else if (i == 0) {
          tgt[sl] = -1;
        }
      }
      if (any) {
#pragma unroll
        for (int q = 0; q < GC; ++q) u[(size_t)row * GC + q] = acc[q];
      }
    }
    __syncthreads();
    // stage 2: out[n][c] = sum over contributing sites and the n half of conj(P_n) u
    {
      const int wv = t >> 6;
      cplx<T> acc[CPT];
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[q] = mk<T>(0, 0);
      for (int n = t & 63; n < d2; n += 64) {
        const int s = n / nv, iv = n - s * nv;
#pragma unroll
        for (int q = 0; q < CPT; ++q) acc[q] = mk<T>(0, 0);
        for (int sl = 0; sl < na; ++sl) {
          const long ts = tgt[sl];
          if (ts < 0) continue;
          const SP<S>* Pi = P + (long)iv * vs + ts * d + s * hd;
          const cplx<T>* uu = u + ((size_t)sl * d + s * hd) * GC + wv * CPT;
          for (int k = 0; k < hd; ++k) {
            const cplx<T> pv = Store<S>::template ld<T>(Pi + k);
#pragma unroll
            for (int q = 0; q < CPT; ++q) cfmac(acc[q], pv, uu[k * GC + q]);
          }
        }
        long recv = Y;
        if (part > 0) {
          int yc[4];
          long b = Y;
          yc[0] = (int)(b % a.NA[0]); b /= a.NA[0];
          yc[1] = (int)(b % a.NA[1]); b /= a.NA[1];
          yc[2] = (int)(b % a.NA[2]);
          yc[3] = (int)(b / a.NA[2]);
          recv = coarse_neighbour(g2, yc, mu, -step);
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int jv = jv0 + wv * CPT + q;
          if (jv < nv) Store<S>::st(Dc2 + ((recv * 9 + part) * (long)d2 + sp * nv + jv) * d2 + n, acc[q]);
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, typename S>
void launch_galerkin_coarse(const CoarseGeom& g, int d, const int agg[4], const SP<S>* Dc1, const SP<S>* P, int nv,
                            SP<S>* Dc2, hipStream_t st) {
  CAgg a = make_cagg(g, agg);
  CoarseGeom g2;
  g2.V = 1;
  for (int m = 0; m < 4; ++m) { g2.L[m] = a.NA[m]; g2.V *= a.NA[m]; }
  const size_t shc = (size_t)a.na * (d / 2 + d) * GAL_GC * sizeof(cplx<T>) + a.na * sizeof(long);
  if (shc <= 150 * 1024) {
    static bool attr = false;   // per instantiation: raise the dynamic LDS limit once
    if (!attr && shc > 64 * 1024) {
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_galerkin_coarse_cols<T, S>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
      attr = true;
    }
    hipLaunchKernelGGL((k_galerkin_coarse_cols<T, S>), dim3((unsigned)g2.V, 2, (nv + GAL_GC - 1) / GAL_GC),
                       dim3(256), shc, st, g, d, a, Dc1, P, nv, Dc2, g2);
    return;
  }
  size_t sh = 2 * (size_t)a.na * d * sizeof(cplx<T>) + a.na * sizeof(long) + 256 * sizeof(cplx<T>);
  hipLaunchKernelGGL((k_galerkin_coarse<T, S>), dim3((unsigned)g2.V, 2 * nv), dim3(256), sh, st, g, d, a, Dc1, P, nv,
                     Dc2, g2);
}

#define INST_TS(T, S)                                                                                              \
  template void launch_coarse_apply<T, S>(const CoarseGeom&, int, const SP<S>*, const cplx<T>*, cplx<T>*, int,     \
                                          const double*, hipStream_t);                                             \
  template void launch_sap_coarse<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, const cplx<T>*,          \
                                        cplx<T>*, int, const double*, const int*, int, int, hipStream_t);          \
  template void launch_restrict_coarse<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, int,                \
                                             const cplx<T>*, cplx<T>*, int, hipStream_t);                          \
  template void launch_prolong_coarse<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, int, const cplx<T>*, \
                                            cplx<T>*, int, hipStream_t);                                           \
  template void launch_gs_coarse<T, S>(const CoarseGeom&, int, const int*, const cplx<T>*, int, cplx<double>*,     \
                                       SP<S>*, hipStream_t);                                                       \
  template void launch_galerkin_coarse<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, const SP<S>*, int,  \
                                             SP<S>*, hipStream_t);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(float, __hip_bfloat16)
INST_TS(float, __half)
template void launch_gamma5_coarse<double>(long, int, const cplx<double>*, cplx<double>*, int, hipStream_t);
template void launch_gamma5_coarse<float>(long, int, const cplx<float>*, cplx<float>*, int, hipStream_t);
