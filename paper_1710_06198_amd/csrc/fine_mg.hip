// Fine-level multigrid kernels: restriction P^dag and prolongation P between
// the fine lattice and the first coarse level, block Gram-Schmidt of the
// fine test vectors, and the Galerkin coarse operator D_c = P^dag D P
// (Sec. 1.1).  Aggregates are the blocks of the fine site ordering.
#include "kernels.h"
#include "su3.h"

template <typename S> using SP = typename Store<S>::pair;

// ------------------------------------------------------------------ restriction (K4)
// One workgroup per aggregate (one thread per site):
// out(y, s*nv + i) = sum_{x in y} sum_{k in s} conj(P_i[k](x)) in[k](x)
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_restrict_fine(FineGeom g, const SP<S>* __restrict__ P, int nv,
                                                       const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* red = reinterpret_cast<cplx<T>*>(smem_raw);   // [nwaves][2nv]
  const long V = g.V;
  const int y = blockIdx.x, r = blockIdx.y;
  const long s = (long)y * g.bvol + threadIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int no = 2 * nv;
  cplx<T> f[12];
  const size_t ts = tsite((unsigned)s, 12);
  const cplx<T>* inr = in + (long)r * 12 * V + ts;
#pragma unroll
  for (int k = 0; k < 12; ++k) f[k] = inr[k * FT];
  for (int i = 0; i < nv; ++i) {
    const SP<S>* Pi = P + (long)i * 12 * V + ts;
    cplx<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
#pragma unroll
    for (int k = 0; k < 6; ++k) cfmac(a0, Store<S>::template ld<T>(Pi + k * FT), f[k]);
#pragma unroll
    for (int k = 6; k < 12; ++k) cfmac(a1, Store<S>::template ld<T>(Pi + k * FT), f[k]);
    a0.re = wave_sum(a0.re); a0.im = wave_sum(a0.im);
    a1.re = wave_sum(a1.re); a1.im = wave_sum(a1.im);
    if (lane == 0) { red[w * no + i] = a0; red[w * no + nv + i] = a1; }
  }
  __syncthreads();
  if (threadIdx.x < no) {
    cplx<T> sum = mk<T>(0, 0);
    for (int k = 0; k < nw; ++k) sum += red[k * no + threadIdx.x];
    out[((long)r * g.nblocks + y) * no + threadIdx.x] = sum;
  }
}
template <typename T, typename S>
void launch_restrict_fine(const FineGeom& g, const SP<S>* P, int nv, const cplx<T>* in, cplx<T>* out, int nrhs,
                          hipStream_t st) {
  size_t sh = (size_t)(g.bvol / 64) * 2 * nv * sizeof(cplx<T>);
  hipLaunchKernelGGL((k_restrict_fine<T, S>), dim3(g.nblocks, nrhs), dim3(g.bvol), sh, st, g, P, nv, in, out);
}

// ------------------------------------------------------------------ prolongation (K5)
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_prolong_fine(FineGeom g, const SP<S>* __restrict__ P, int nv,
                                                      const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* e = reinterpret_cast<cplx<T>*>(smem_raw);
  const long V = g.V;
  const int y = blockIdx.x, r = blockIdx.y;
  const int no = 2 * nv;
  for (int k = threadIdx.x; k < no; k += blockDim.x) e[k] = in[((long)r * g.nblocks + y) * no + k];
  __syncthreads();
  const long s = (long)y * g.bvol + threadIdx.x;
  const size_t ts = tsite((unsigned)s, 12);
  cplx<T> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<T>(0, 0);
  for (int i = 0; i < nv; ++i) {
    const SP<S>* Pi = P + (long)i * 12 * V + ts;
    cplx<T> e0 = e[i], e1 = e[nv + i];
#pragma unroll
    for (int k = 0; k < 6; ++k) cfma(acc[k], Store<S>::template ld<T>(Pi + k * FT), e0);
#pragma unroll
    for (int k = 6; k < 12; ++k) cfma(acc[k], Store<S>::template ld<T>(Pi + k * FT), e1);
  }
  cplx<T>* o = out + (long)r * 12 * V + ts;
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k * FT] = acc[k];
}
template <typename T, typename S>
void launch_prolong_fine(const FineGeom& g, const SP<S>* P, int nv, const cplx<T>* in, cplx<T>* out, int nrhs,
                         hipStream_t st) {
  size_t sh = (size_t)2 * nv * sizeof(cplx<T>);
  hipLaunchKernelGGL((k_prolong_fine<T, S>), dim3(g.nblocks, nrhs), dim3(g.bvol), sh, st, g, P, nv, in, out);
}

// ------------------------------------------------------------------ block Gram-Schmidt (K7)
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_gs_fine(FineGeom g, const cplx<T>* __restrict__ tv, int nv,
                                                 cplx<double>* P64, SP<S>* P) {
  __shared__ double red[4][2 * 64];
  const long V = g.V;
  const int y = blockIdx.x, sc = blockIdx.y;   // aggregate, chirality
  const long s = (long)y * g.bvol + threadIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const long vs = 12 * V;
  const size_t base = tsite((unsigned)s, 12) + (size_t)sc * 6 * FT;
  for (int i = 0; i < nv; ++i) {
    cplx<double> x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cplx<T> v = tv[(long)i * vs + base + k * FT];
      x[k] = mk((double)v.re, (double)v.im);
    }
    for (int pass = 0; pass < 2 && i > 0; ++pass) {
      for (int j0 = 0; j0 < i; j0 += 64) {
        int nj = min(64, i - j0);
        for (int jj = 0; jj < nj; ++jj) {
          cplx<double> p = mk(0.0, 0.0);
          const cplx<double>* q = P64 + (long)(j0 + jj) * vs + base;
#pragma unroll
          for (int k = 0; k < 6; ++k) cfmac(p, q[k * FT], x[k]);
          p.re = wave_sum(p.re);
          p.im = wave_sum(p.im);
          if (lane == 0) { red[w][2 * jj] = p.re; red[w][2 * jj + 1] = p.im; }
        }
        __syncthreads();
        for (int jj = 0; jj < nj; ++jj) {
          cplx<double> cj = mk(0.0, 0.0);
          for (int ww = 0; ww < nw; ++ww) cj += mk(red[ww][2 * jj], red[ww][2 * jj + 1]);
          const cplx<double>* q = P64 + (long)(j0 + jj) * vs + base;
#pragma unroll
          for (int k = 0; k < 6; ++k) x[k] -= cj * q[k * FT];
        }
        __syncthreads();
      }
    }
    double nn = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) nn += norm2(x[k]);
    nn = wave_sum(nn);
    if (lane == 0) red[w][0] = nn;
    __syncthreads();
    nn = 0;
    for (int ww = 0; ww < nw; ++ww) nn += red[ww][0];
    __syncthreads();
    double inv = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cplx<double> q = inv * x[k];
      P64[(long)i * vs + base + k * FT] = q;
      Store<S>::st(P + (long)i * vs + base + k * FT, q);
    }
  }
}
template <typename T, typename S>
void launch_gs_fine(const FineGeom& g, const cplx<T>* tv, int nv, cplx<double>* P64, SP<S>* P, hipStream_t st) {
  hipLaunchKernelGGL((k_gs_fine<T, S>), dim3(g.nblocks, 2), dim3(g.bvol), 0, st, g, tv, nv, P64, P);
}

// ------------------------------------------------------------------ Galerkin (K8), fine -> first coarse level
// Workgroup per (aggregate y, coarse column cc = s'*nv + j), one thread per
// site.  w = column cc of P on y.  Part 0: the aggregate-internal part of D
// (clover + hops that stay in y) gives D_c[y][0][cc].  Part 1+2mu: forward
// hops from sites x' = x - mu outside y's lower face pull w(x); they land in
// y - mu's block 1+2mu.  Part 2+2mu: backward hops at x'' = x + mu from y's
// upper face land in y + mu's block 2+2mu.
template <int MU, typename T>
TM_D void lds_spinor(const cplx<T>* wl, int bv, int sp, int nl, cplx<T>* pn) {
#pragma unroll
  for (int k = 0; k < 12; ++k) pn[k] = (k / 6 == sp) ? wl[(k % 6) * bv + nl] : mk<T>(0, 0);
}

template <int MU, typename T>
TM_D void intra_hops(const FineOp<T>& op, const cplx<T>* wl, int sp, long s, int loc, const int c[4], cplx<T>* acc) {
  const FineGeom& g = op.g;
  const int bv = g.bvol;
  const int lc = c[MU] % g.B[MU];
  cplx<T> pn[12];
  if (lc < g.B[MU] - 1) {
    lds_spinor<MU>(wl, bv, sp, loc + g.lstride[MU], pn);
    M3<T> u = load_link(op.links, MU, s, g.V);
    hop_fwd<MU>(u, pn, acc);
  }
  if (lc > 0) {
    lds_spinor<MU>(wl, bv, sp, loc - g.lstride[MU], pn);
    M3<T> ub = load_link(op.links, MU, s - g.lstride[MU], g.V);
    hop_bwd<MU>(ub, pn, acc);
  }
}

template <int MU, typename T>
TM_D bool face_hop(const FineOp<T>& op, int step, long s, const int c[4], const cplx<T>* wx, cplx<T>* v, long& tgt_site) {
  const FineGeom& g = op.g;
  const int lc = c[MU] % g.B[MU];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = mk<T>(0, 0);
  if (step > 0) {
    if (lc != 0) return false;
    tgt_site = fine_neighbour(g, s, c, MU, -1);      // x' = x - mu, forward hop at x' pulls w(x)
    M3<T> u = load_link(op.links, MU, tgt_site, g.V);
    hop_fwd<MU>(u, wx, v);
  } else {
    if (lc != g.B[MU] - 1) return false;
    tgt_site = fine_neighbour(g, s, c, MU, +1);      // x'' = x + mu, backward hop at x'' pulls w(x)
    M3<T> u = load_link(op.links, MU, s, g.V);
    hop_bwd<MU>(u, wx, v);
  }
  return true;
}

// LDS: w (the column's chirality half, 6 x bv), u (one chirality half of the
// pushed vectors, 6 x bv), the receiving site of every source, a reduction
// buffer: 48 bv + 8 bv + 4 KB bytes in FP64 (54 KB for 256-site aggregates).
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_galerkin_fine(FineOp<T> op, const SP<S>* __restrict__ P, int nv,
                                                       SP<S>* Dc) {
  extern __shared__ unsigned char smem_raw[];
  const FineGeom& g = op.g;
  const long V = g.V;
  const int bv = g.bvol;
  cplx<T>* wl = reinterpret_cast<cplx<T>*>(smem_raw);   // [6][bv]
  cplx<T>* u = wl + 6 * bv;                             // [6][bv]
  long* tgt = reinterpret_cast<long*>(u + 6 * bv);     // [bv]
  cplx<T>* red = reinterpret_cast<cplx<T>*>(tgt + bv); // [256]
  const int y = blockIdx.x, cc = blockIdx.y;
  const int sp = cc / nv, jv = cc - sp * nv;
  const int loc = threadIdx.x;
  const long s = (long)y * bv + loc;
  const int no = 2 * nv;
  int c[4];
  fine_coords(g, s, c);
  cplx<T> wx[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    bool in_s = (k < 6) == (sp == 0);
    wx[k] = in_s ? Store<S>::template ld<T>(P + (long)jv * 12 * V + tsite((unsigned)s, 12) + k * FT) : mk<T>(0, 0);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) wl[k * bv + loc] = wx[sp * 6 + k];
  __syncthreads();
  int yc[4];
  {
    int b = y;
    yc[0] = b % g.NB[0]; b /= g.NB[0];
    yc[1] = b % g.NB[1]; b /= g.NB[1];
    yc[2] = b % g.NB[2];
    yc[3] = b / g.NB[2];
  }
  for (int part = 0; part < 9; ++part) {
    cplx<T> v[12];
    long ts = -1;
    if (part == 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = mk<T>(0, 0);
      clover_block_mv(op.clover, (unsigned)s, V, wx, v);
      clover_block_mv(op.clover + 36 * V, (unsigned)s, V, wx + 6, v + 6);
      intra_hops<0>(op, wl, sp, s, loc, c, v);
      intra_hops<1>(op, wl, sp, s, loc, c, v);
      intra_hops<2>(op, wl, sp, s, loc, c, v);
      intra_hops<3>(op, wl, sp, s, loc, c, v);
      ts = s;
    } else {
      const int mu = (part - 1) >> 1;
      const int step = ((part - 1) & 1) ? -1 : 1;
      bool on = false;
      switch (mu) {
        case 0: on = face_hop<0>(op, step, s, c, wx, v, ts); break;
        case 1: on = face_hop<1>(op, step, s, c, wx, v, ts); break;
        case 2: on = face_hop<2>(op, step, s, c, wx, v, ts); break;
        default: on = face_hop<3>(op, step, s, c, wx, v, ts); break;
      }
      if (!on) ts = -1;
    }
    tgt[loc] = ts;
    long recv = y;
    if (part > 0) {
      const int mu = (part - 1) >> 1;
      const int step = ((part - 1) & 1) ? -1 : 1;
      int rc[4] = {yc[0], yc[1], yc[2], yc[3]};
      rc[mu] = (rc[mu] - step + g.NB[mu]) % g.NB[mu];
      recv = ((long)(rc[3] * g.NB[2] + rc[2]) * g.NB[1] + rc[1]) * g.NB[0] + rc[0];
    }
    // project onto P at the receiving sites, one chirality at a time
    for (int sc = 0; sc < 2; ++sc) {
#pragma unroll
      for (int k = 0; k < 6; ++k) u[k * bv + loc] = v[sc * 6 + k];
      __syncthreads();
      const int G = max(1, (int)blockDim.x / nv);
      const int t = threadIdx.x, iv = t % nv, grp = t / nv;
      cplx<T> acc = mk<T>(0, 0);
      if (grp < G) {
        const SP<S>* Pi = P + (long)iv * 12 * V + (long)sc * 6 * FT;
        for (int l = grp; l < bv; l += G) {
          long tsl = tgt[l];
          if (tsl < 0) continue;
#pragma unroll
          for (int k = 0; k < 6; ++k)
            cfmac(acc, Store<S>::template ld<T>(Pi + tsite((unsigned)tsl, 12) + k * FT), u[k * bv + l]);
        }
      }
      red[t] = acc;
      __syncthreads();
      if (t < nv) {
        cplx<T> sum = mk<T>(0, 0);
        for (int k = 0; k < G; ++k) sum += red[k * nv + t];
        Store<S>::st(Dc + ((recv * 9 + part) * (long)no + cc) * no + sc * nv + t, sum);
      }
      __syncthreads();
    }
  }
}
template <typename T, typename S>
void launch_galerkin_fine(const FineOp<T>& op, const SP<S>* P, int nv, SP<S>* Dc, hipStream_t st) {
  const int bv = op.g.bvol;
  size_t sh = 12 * (size_t)bv * sizeof(cplx<T>) + bv * sizeof(long) + 256 * sizeof(cplx<T>);
  hipLaunchKernelGGL((k_galerkin_fine<T, S>), dim3(op.g.nblocks, 2 * nv), dim3(bv), sh, st, op, P, nv, Dc);
}

// ------------------------------------------------------------------ noise
TM_D unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
template <typename T>
__global__ void k_random(cplx<T>* out, long count, unsigned long long seed) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= count) return;
  unsigned long long h1 = mix64(seed * 0x632BE59BD9B4E019ULL + 2 * (unsigned long long)k);
  unsigned long long h2 = mix64(h1 ^ (2 * (unsigned long long)k + 1));
  double u1 = ((double)(h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  double u2 = ((double)(h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  double rad = sqrt(-log(u1));
  double ph = 6.283185307179586 * u2;
  out[k] = mk<T>((T)(rad * cos(ph)), (T)(rad * sin(ph)));
}
template <typename T>
void launch_random(cplx<T>* out, long count, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(k_random<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, out, count, seed);
}

template <typename S>
__global__ void k_store_to64(const SP<S>* in, cplx<double>* out, long count) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k < count) out[k] = Store<S>::template ld<double>(in + k);
}
template <typename S>
__global__ void k_store_from64(const cplx<double>* in, SP<S>* out, long count) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k < count) Store<S>::st(out + k, in[k]);
}
template <typename S>
void launch_store_to64(const SP<S>* in, cplx<double>* out, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_store_to64<S>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, in, out, count);
}
template <typename S>
void launch_store_from64(const cplx<double>* in, SP<S>* out, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_store_from64<S>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, in, out, count);
}

#define INST_TS(T, S)                                                                                            \
  template void launch_restrict_fine<T, S>(const FineGeom&, const SP<S>*, int, const cplx<T>*, cplx<T>*, int,    \
                                           hipStream_t);                                                         \
  template void launch_prolong_fine<T, S>(const FineGeom&, const SP<S>*, int, const cplx<T>*, cplx<T>*, int,     \
                                          hipStream_t);                                                          \
  template void launch_gs_fine<T, S>(const FineGeom&, const cplx<T>*, int, cplx<double>*, SP<S>*, hipStream_t);  \
  template void launch_galerkin_fine<T, S>(const FineOp<T>&, const SP<S>*, int, SP<S>*, hipStream_t);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(float, __hip_bfloat16)
INST_TS(float, __half)
template void launch_random<double>(cplx<double>*, long, unsigned long long, hipStream_t);
template void launch_random<float>(cplx<float>*, long, unsigned long long, hipStream_t);
#define INST_S(S)                                                                         \
  template void launch_store_to64<S>(const SP<S>*, cplx<double>*, long, hipStream_t);     \
  template void launch_store_from64<S>(const cplx<double>*, SP<S>*, long, hipStream_t);
INST_S(double)
INST_S(float)
INST_S(__hip_bfloat16)
INST_S(__half)
