// Fine-level multigrid kernels: restriction P^dag and prolongation P between
// the fine lattice and the first coarse level, block Gram-Schmidt of the
// fine test vectors, and the Galerkin coarse operator D_c = P^dag D P
// (Sec. 1.1).  Aggregates are the blocks of the fine site ordering.
#include <type_traits>

#include "kernels.h"
#include "mfma.h"
#include "solver.h"
#include "su3.h"

template <typename S> using SP = typename Store<S>::pair;

constexpr int GPM_TS = 16;   // sites per LDS tile of the matrix-core products

// ------------------------------------------------------------------ batched transfers on the matrix cores
// With 8 or more right-hand sides (FP32 vectors, bf16 P, N_v <= 32) the
// transfers are dense products over an aggregate, 16 right-hand sides per
// workgroup:
//   P^dag:  out[(s, i)][r] = sum_{x, k in s} conj(P_i(x)_k) in_r(x)_k,
//           per chirality an (N_v x 1536) x (1536 x 16) product;
//   P:      out_r(x)_k     = sum_i P_i(x)_k e_r[(s(k), i)],
//           a (3072 x N_v) x (N_v x 16) product.
// P is exact in bf16; the FP32 vectors are split into two bf16 parts (kept
// to 2^-18 of their size); 16x16x32 bf16 MFMA tiles, FP32 accumulation.
constexpr int TR_NR = 16;

TM_D bool tr_unit(const FineGeom& g, int nrhs, int& y, int& r0) {
  // workgroup -> (aggregate, group of 16 right-hand sides), the groups of
  // one aggregate on one XCD back to back
  const int ng = (nrhs + TR_NR - 1) / TR_NR;
  const int x8 = blockIdx.x & 7, rest = blockIdx.x >> 3;
  r0 = (rest % ng) * TR_NR;
  y = (rest / ng) * 8 + x8;
  return y < g.nblocks;
}

__global__ void __launch_bounds__(256) k_restrict_mf(FineGeom g, const bf16pair* __restrict__ P, int nv,
                                                     const cplx<float>* __restrict__ in, cplx<float>* __restrict__ out,
                                                     int nrhs) {
  int y, r0;
  if (!tr_unit(g, nrhs, y, r0)) return;
  const long V = g.V;
  const int no = 2 * nv;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  const int sc = wv >> 1, mt = wv & 1;   // chirality and row (vector) tile of this wave
  const int iv = 16 * mt + lr, r = r0 + lr;
  const unsigned* Pu = reinterpret_cast<const unsigned*>(P);
  // K steps: component k of chirality sc, 16 consecutive sites; lane group
  // lk holds sites 4 lk .. 4 lk + 3, one 16-byte load of P and two of the
  // input per step, straight from memory (no LDS, no barrier)
  const unsigned* pbase = Pu + (long)(iv < nv ? iv : 0) * 12 * V;
  const cplx<float>* ibase = in + (long)(r < nrhs ? r : r0) * 12 * V;
  mf_f4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  const int nxt = g.bvol / 16;
  for (int step = 0; step < 6 * nxt; ++step) {
    const int kk = step / nxt, xb = step - kk * nxt, k = 6 * sc + kk;
    const size_t o = tsite((unsigned)((long)y * g.bvol + 16 * xb + 4 * lk), 12) + k * FT;
    uint4 pu = make_uint4(0u, 0u, 0u, 0u);
    if (iv < nv) pu = *reinterpret_cast<const uint4*>(pbase + o);
    float4 z01 = make_float4(0.f, 0.f, 0.f, 0.f), z23 = z01;
    if (r < nrhs) {
      z01 = reinterpret_cast<const float4*>(ibase + o)[0];
      z23 = reinterpret_cast<const float4*>(ibase + o)[1];
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
    // Re(conj(P) z) = Re P Re z + Im P Im z, Im(conj(P) z) = Re P Im z - Im P Re z
    mf_cmac_conj(ar, ai, bb, accr, acci);
  }
  // C tile: lane l holds rows (vectors) 16 mt + 4 (l / 16) + v, column (rhs) l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int ivo = 16 * mt + 4 * lk + v, rr = r0 + lr;
    if (ivo < nv && rr < nrhs) out[((long)rr * g.nblocks + y) * no + sc * nv + ivo] = mk(accr[v], acci[v]);
  }
}

__global__ void __launch_bounds__(256) k_prolong_mf(FineGeom g, const bf16pair* __restrict__ P, int nv,
                                                    const cplx<float>* __restrict__ in, cplx<float>* __restrict__ out,
                                                    int nrhs) {
  __shared__ cplx<float> ev[TR_NR * 64];          // [rhs][s nv + i], nv <= 32
  __shared__ cplx<float> sb[4][TR_NR * 16];       // per wave: [rhs][site of the tile]
  int y, r0;
  if (!tr_unit(g, nrhs, y, r0)) return;
  const long V = g.V;
  const int no = 2 * nv;
  const int t = threadIdx.x, wv = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  for (int e = t; e < TR_NR * no; e += 256) {
    const int j = e / no, i = e - j * no;
    ev[j * 64 + i] = r0 + j < nrhs ? in[((long)(r0 + j) * g.nblocks + y) * no + i] : mk<float>(0, 0);
  }
  __syncthreads();
  const unsigned* Pu = reinterpret_cast<const unsigned*>(P);
  const int nxt = g.bvol / 16;   // 16-site tiles of the aggregate
  // row tiles (component k, 16 consecutive sites); wave wv takes every fourth
  for (int tile = wv; tile < 12 * nxt; tile += 4) {
    const int k = tile / nxt, xb = tile - k * nxt, sc = k / 6;
    const size_t ts = tsite((unsigned)((long)y * g.bvol + 16 * xb + lr), 12) + k * FT;
    mf_f4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
    for (int i0 = 0; i0 < nv; i0 += 16) {
      mf_s4 ar, ai;
      cplx<float> bv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + 4 * lk + e;
        const unsigned u = i < nv ? Pu[(long)i * 12 * V + ts] : 0u;
        ar[e] = (short)(u & 0xffffu);
        ai[e] = (short)(u >> 16);
        bv[e] = i < nv ? ev[lr * 64 + sc * nv + i] : mk<float>(0, 0);
      }
      const MfSplit bb = mf_split(bv);
      // Re(P e) = Re P Re e - Im P Im e, Im(P e) = Re P Im e + Im P Re e
      mf_cmac(ar, ai, bb, accr, acci);
    }
    // C: lane l holds sites 4 (l / 16) + v of the tile for rhs l % 16; staged
    // in LDS so that each lane stores four consecutive sites of one rhs
#pragma unroll
    for (int v = 0; v < 4; ++v) sb[wv][lr * 16 + 4 * lk + v] = mk(accr[v], acci[v]);
    __builtin_amdgcn_wave_barrier();
    {
      const int j = l >> 2, xq = 4 * (l & 3), r = r0 + j;
      if (r < nrhs) {
        cplx<float>* o = out + (long)r * 12 * V + tsite((unsigned)((long)y * g.bvol + 16 * xb + xq), 12) + k * FT;
        const float4 a = make_float4(sb[wv][j * 16 + xq].re, sb[wv][j * 16 + xq].im, sb[wv][j * 16 + xq + 1].re,
                                     sb[wv][j * 16 + xq + 1].im);
        const float4 b = make_float4(sb[wv][j * 16 + xq + 2].re, sb[wv][j * 16 + xq + 2].im,
                                     sb[wv][j * 16 + xq + 3].re, sb[wv][j * 16 + xq + 3].im);
        reinterpret_cast<float4*>(o)[0] = a;
        reinterpret_cast<float4*>(o)[1] = b;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------------ restriction (K4)
// One workgroup per aggregate (one thread per site):
// out(y, s*nv + i) = sum_{x in y} sum_{k in s} conj(P_i[k](x)) in[k](x)
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_restrict_fine(FineGeom g, const SP<S>* __restrict__ P, int nv,
                                                       const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                       int nrhs) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* red = reinterpret_cast<cplx<T>*>(smem_raw);   // [nwaves][2nv]
  const long V = g.V;
  // workgroup -> (aggregate, rhs): the right-hand sides of one aggregate run
  // on one XCD back to back, so its rows of P come from that L2 after the
  // first; with one right-hand side this is the identity
  const int x8 = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int r = rest % nrhs, y = (rest / nrhs) * 8 + x8;
  if (y >= g.nblocks) return;
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
  const unsigned n8 = (unsigned)((g.nblocks + 7) / 8 * 8);
  if constexpr (std::is_same<T, float>::value && std::is_same<S, __hip_bfloat16>::value) {
    const int tv = tune_get(TUNE_RESTRICT0, nv, g.V, nrhs);
    if ((tv >= 0 ? tv == 1 : nrhs >= 8) && nv <= 32 && g.bvol % 16 == 0) {
      hipLaunchKernelGGL(k_restrict_mf, dim3(n8 * ((nrhs + TR_NR - 1) / TR_NR)), dim3(256), 0, st, g, P, nv, in, out,
                         nrhs);
      tune_used(TUNE_RESTRICT0, 1);
      return;
    }
  }
  tune_used(TUNE_RESTRICT0, 0);
  hipLaunchKernelGGL((k_restrict_fine<T, S>), dim3(n8 * nrhs), dim3(g.bvol), sh, st, g, P, nv, in, out, nrhs);
}

// ------------------------------------------------------------------ prolongation (K5)
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_prolong_fine(FineGeom g, const SP<S>* __restrict__ P, int nv,
                                                      const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                      int nrhs) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* e = reinterpret_cast<cplx<T>*>(smem_raw);
  const long V = g.V;
  // workgroup -> (aggregate, rhs): the right-hand sides of one aggregate run
  // on one XCD back to back, so its rows of P come from that L2 after the
  // first; with one right-hand side this is the identity
  const int x8 = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int r = rest % nrhs, y = (rest / nrhs) * 8 + x8;
  if (y >= g.nblocks) return;
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
  const unsigned n8 = (unsigned)((g.nblocks + 7) / 8 * 8);
  if constexpr (std::is_same<T, float>::value && std::is_same<S, __hip_bfloat16>::value) {
    const int tv = tune_get(TUNE_PROLONG0, nv, g.V, nrhs);
    if ((tv >= 0 ? tv == 1 : nrhs >= 8) && nv <= 32 && g.bvol % 16 == 0) {
      hipLaunchKernelGGL(k_prolong_mf, dim3(n8 * ((nrhs + TR_NR - 1) / TR_NR)), dim3(256), 0, st, g, P, nv, in, out,
                         nrhs);
      tune_used(TUNE_PROLONG0, 1);
      return;
    }
  }
  tune_used(TUNE_PROLONG0, 0);
  hipLaunchKernelGGL((k_prolong_fine<T, S>), dim3(n8 * nrhs), dim3(g.bvol), sh, st, g, P, nv, in, out, nrhs);
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
// Cholesky QR, twice (CholQR2), for up to 32 vectors: per (aggregate,
// chirality) workgroup the K = 6 * bvol rows of V = [v_1 .. v_nv] give the
// Gram matrix G1 = V^dag V (FP64, accumulated from LDS tiles of rows), its
// Cholesky factor G1 = R1^dag R1 (positive real diagonal) and Q1 = V R1^-1;
// the second pass takes the Gram matrix of Q1 (formed tile by tile from V,
// never stored), its factor R2, and the result is Q = V (R1^-1 R2^-1).
// Given the same v_i this is the Q of Gram-Schmidt in index order (the QR
// factor with positive diagonal is unique); it reads V three times and
// needs a handful of barriers instead of a chain of nv^2 dependent
// reductions.
constexpr int GS_NV = 32;   // largest nv of the Cholesky QR kernel
constexpr int GS_TS = 8;    // sites per LDS tile
constexpr int GS_NR = GS_TS * 6 / 2;   // row pairs per tile

// Tiles hold nvp = nv rounded up to 4 columns (the padding columns are
// zero), rows (site in tile, component) as xs * 6 + k, row stride nvp + 1
// (an odd stride keeps the lanes of a tile load in different LDS banks).
TM_D int gs_nvp(int nv) { return (nv + 3) & ~3; }

// A tile is fetched into registers (GS_EPT values per thread) while the
// previous one is processed, then stored to LDS: the global latency of the
// next tile overlaps the arithmetic on the current one.
constexpr int GS_EPT = (GS_TS * 6 * GS_NV + 255) / 256;

template <typename U>
TM_D void gs_fetch_tile(const cplx<U>* src, long vs, long site0, int x0, int sc, int nv, int nvp,
                        cplx<double> (&reg)[GS_EPT]) {
  const int nrow = GS_TS * 6;
#pragma unroll
  for (int q = 0; q < GS_EPT; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int xs = e % GS_TS, rem = e / GS_TS, k = rem % 6, c = rem / 6;
    reg[q] = mk(0.0, 0.0);
    if (e < nrow * nvp && c < nv) {
      const cplx<U> x = src[(long)c * vs + tsite((unsigned)(site0 + x0 + xs), 12) + (sc * 6 + k) * FT];
      reg[q] = mk((double)x.re, (double)x.im);
    }
  }
}
TM_D void gs_store_tile(int nvp, const cplx<double> (&reg)[GS_EPT], cplx<double>* tile) {
  const int nrow = GS_TS * 6;
#pragma unroll
  for (int q = 0; q < GS_EPT; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int xs = e % GS_TS, rem = e / GS_TS, k = rem % 6, c = rem / 6;
    if (e < nrow * nvp) tile[(xs * 6 + k) * (nvp + 1) + c] = reg[q];
  }
}

// q = rows r0 and r0 + GS_NR of tile x M, columns 4 cg .. 4 cg + 3 (M upper
// triangular nv x nv, so column c sums i <= c)
TM_D void gs_rows_times(const cplx<double>* tile, int nv, int nvp, const cplx<double>* M, int r0, int cg,
                        cplx<double> q[2][4]) {
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) q[h][j] = mk(0.0, 0.0);
  const int iend = min(4 * cg + 4, nv);
  for (int i = 0; i < iend; ++i) {
    const cplx<double> v0 = tile[r0 * (nvp + 1) + i], v1 = tile[(r0 + GS_NR) * (nvp + 1) + i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * cg + j;
      const cplx<double> m = (c < nv && i <= c) ? M[i * nv + c] : mk(0.0, 0.0);
      cfma(q[0][j], v0, m);
      cfma(q[1][j], v1, m);
    }
  }
}

// G = W^dag W over the aggregate's rows, W = V (XF == false) or V M.
// Thread (block, slice): a 4x4 block (ba <= bb) of G over the tile rows
// r = slice (mod nslice), 16 products per 8 values read from LDS; slices
// are summed in slice order at the end.  G: [nv][nv], both triangles.
template <typename U, bool XF>
TM_D void gs_gram(const cplx<U>* src, long vs, long site0, int bvol, int sc, int nv, const cplx<double>* M,
                  cplx<double>* tile, cplx<double>* G) {
  const int t = threadIdx.x, nvp = gs_nvp(nv), nb = nvp / 4;
  const int nblk = nb * (nb + 1) / 2, nslice = 256 / nblk;
  const int nrow = GS_TS * 6;
  const bool active = t < nblk * nslice;
  const int blk = t % nblk, slice = t / nblk;
  int ba = 0, bb = blk;
  while (bb >= nb - ba) { bb -= nb - ba; ++ba; }
  bb += ba;   // blocks (ba, bb), ba <= bb, in row order
  const int r0 = t % GS_NR, cg = t / GS_NR;   // transform mapping
  cplx<double> acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
  cplx<double> reg[GS_EPT];
  gs_fetch_tile<U>(src, vs, site0, 0, sc, nv, nvp, reg);
  for (int x0 = 0; x0 < bvol; x0 += GS_TS) {
    gs_store_tile(nvp, reg, tile);
    __syncthreads();
    if (x0 + GS_TS < bvol) gs_fetch_tile<U>(src, vs, site0, x0 + GS_TS, sc, nv, nvp, reg);
    if constexpr (XF) {
      cplx<double> q[2][4];
      if (cg < nb) gs_rows_times(tile, nv, nvp, M, r0, cg, q);
      __syncthreads();
      if (cg < nb) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int j = 0; j < 4; ++j) tile[(r0 + h * GS_NR) * (nvp + 1) + 4 * cg + j] = q[h][j];
      }
      __syncthreads();
    }
    if (active) {
      for (int r = slice; r < nrow; r += nslice) {
        cplx<double> va[4], vb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          va[i] = tile[r * (nvp + 1) + 4 * ba + i];
          vb[i] = tile[r * (nvp + 1) + 4 * bb + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) cfmac(acc[i][j], va[i], vb[j]);
      }
    }
    __syncthreads();
  }
  for (int sl = 0; sl < nslice; ++sl) {
    if (active && slice == sl) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = 4 * ba + i, b2 = 4 * bb + j;
          if (a < nv && b2 < nv && a <= b2) G[a * nv + b2] = sl == 0 ? acc[i][j] : G[a * nv + b2] + acc[i][j];
        }
    }
    __syncthreads();
  }
  for (int e = t; e < nv * nv; e += blockDim.x) {
    const int a = e / nv, b2 = e % nv;
    if (a > b2) G[e] = conj(G[b2 * nv + a]);
  }
  __syncthreads();
}

// In place G -> R (upper, G = R^dag R, real positive diagonal), then
// Ri = R^-1 (upper).
TM_D void gs_chol_inv(int nv, cplx<double>* G, cplx<double>* Ri) {
  const int t = threadIdx.x;
  for (int j = 0; j < nv; ++j) {
    __syncthreads();   // previous trailing update done
    const double d = sqrt(fmax(G[j * nv + j].re, 1e-300));
    __syncthreads();   // every thread has read the pivot before it is overwritten
    if (t >= j && t < nv) G[j * nv + t] = (1.0 / d) * G[j * nv + t];   // row j of R (t == j gives d)
    __syncthreads();
    // trailing update G[i][l] -= conj(R[j][i]) R[j][l], j < i <= l (upper part only)
    const int nt = nv - j - 1;
    for (int e = t; e < nt * nt; e += blockDim.x) {
      const int i = j + 1 + e / nt, l = j + 1 + e % nt;
      if (l >= i) G[i * nv + l] -= conj(G[j * nv + i]) * G[j * nv + l];
    }
  }
  __syncthreads();
  // R^-1, one column per thread: Ri[j][j] = 1 / R[j][j]; Ri[i][j] = -(sum_{i<k<=j} R[i][k] Ri[k][j]) / R[i][i]
  if (t < nv) {
    const int j = t;
    for (int i = 0; i < nv; ++i) Ri[i * nv + j] = mk(0.0, 0.0);
    Ri[j * nv + j] = mk(1.0 / G[j * nv + j].re, 0.0);
    for (int i = j - 1; i >= 0; --i) {
      cplx<double> s2 = mk(0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) cfma(s2, G[i * nv + k], Ri[k * nv + j]);
      Ri[i * nv + j] = (-1.0 / G[i * nv + i].re) * s2;
    }
  }
  __syncthreads();
}

template <typename T, typename S>
__global__ void __launch_bounds__(256) k_gs_fine_cholqr(FineGeom g, const cplx<T>* __restrict__ tv, int nv,
                                                        SP<S>* __restrict__ P) {
  __shared__ cplx<double> tile[GS_TS * 6 * (GS_NV + 1)];   // rows of nvp <= GS_NV columns, stride nvp + 1
  __shared__ cplx<double> G[GS_NV * GS_NV];
  __shared__ cplx<double> Ra[GS_NV * GS_NV];
  __shared__ cplx<double> Rb[GS_NV * GS_NV];
  const int y = blockIdx.x, sc = blockIdx.y, t = threadIdx.x;
  const long vs = 12 * g.V, site0 = (long)y * g.bvol;
  const int nvp = gs_nvp(nv), nb = nvp / 4;
  gs_gram<T, false>(tv, vs, site0, g.bvol, sc, nv, nullptr, tile, G);   // V^dag V
  gs_chol_inv(nv, G, Ra);                                               // Ra = R1^-1
  gs_gram<T, true>(tv, vs, site0, g.bvol, sc, nv, Ra, tile, G);         // Q1^dag Q1
  gs_chol_inv(nv, G, Rb);                                               // Rb = R2^-1
  // G = Ra Rb (upper triangular), the column transform taking V to Q
  for (int e = t; e < nv * nv; e += 256) {
    const int i = e / nv, c = e % nv;
    cplx<double> s2 = mk(0.0, 0.0);
    for (int l = i; l <= c; ++l) cfma(s2, Ra[i * nv + l], Rb[l * nv + c]);
    G[e] = s2;
  }
  __syncthreads();
  const int r0 = t % GS_NR, cg = t / GS_NR;
  cplx<double> reg[GS_EPT];
  gs_fetch_tile<T>(tv, vs, site0, 0, sc, nv, nvp, reg);
  for (int x0 = 0; x0 < g.bvol; x0 += GS_TS) {
    gs_store_tile(nvp, reg, tile);
    __syncthreads();
    if (x0 + GS_TS < g.bvol) gs_fetch_tile<T>(tv, vs, site0, x0 + GS_TS, sc, nv, nvp, reg);
    if (cg < nb) {
      cplx<double> q[2][4];
      gs_rows_times(tile, nv, nvp, G, r0, cg, q);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + h * GS_NR, xs = r / 6, k = r % 6;
        const size_t o0 = tsite((unsigned)(site0 + x0 + xs), 12) + (sc * 6 + k) * FT;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = 4 * cg + j;
          if (c < nv) Store<S>::st(P + (size_t)c * vs + o0, q[h][j]);
        }
      }
    }
    __syncthreads();
  }
}

// The Cholesky QR path needs no FP64 copy of the vectors; the sequential
// Gram-Schmidt fallback (more than GS_NV vectors) keeps its pieces in one.
bool gs_fine_needs_fp64_copy(int nv) { return nv > GS_NV; }

template <typename T, typename S>
void launch_gs_fine(const FineGeom& g, const cplx<T>* tv, int nv, cplx<double>* P64, SP<S>* P, hipStream_t st) {
  if (nv <= GS_NV)
    hipLaunchKernelGGL((k_gs_fine_cholqr<T, S>), dim3(g.nblocks, 2), dim3(256), 0, st, g, tv, nv, P);
  else
    hipLaunchKernelGGL((k_gs_fine<T, S>), dim3(g.nblocks, 2), dim3(g.bvol), 0, st, g, tv, nv, P64, P);
}

// ------------------------------------------------------------------ Galerkin, fine -> first coarse level
// D_c = P^dag D P, block by block: D_c[r][part] (part 0 self, 1+2mu the
// neighbour r+mu, 2+2mu the neighbour r-mu) = sum over the sites x of the
// receiving aggregate r of P(x)^dag Z_part(x), with
//   Z_0(x)      = A(x) P_r(x) + hops of D from x to sites of r,
//   Z_{mu,+}(x) = hop of D from x to x+mu, for x on r's upper mu face,
//   Z_{mu,-}(x) = hop of D from x to x-mu, for x on r's lower mu face,
// where P_r is P restricted to aggregate r (all 2 N_v columns).
// Two kernels per chunk of CB columns:
//   k_galerkin_z    one workgroup per (source aggregate y, column), one
//                   thread per site: applies D to the column and writes every
//                   piece to the receiving aggregate's slot in Z;
//   k_galerkin_proj one workgroup per (receiving aggregate, part): the
//                   (2N_v x CB) block P^dag Z, sites in LDS tiles.
// Z layout: [aggregate][part][column in chunk][12][site of the part's
// region], regions of bvol (self) and bvol / B_mu (faces) sites.  Both
// kernels map workgroups so that all work of one aggregate runs on one XCD.
struct GalerkinZ {
  int regoff[9];   // site offset of each part's region in an aggregate's slot
  int regsz[9];    // sites per region
  int za;          // sites per aggregate slot (sum of regsz)
  int c0, cb;      // column chunk
};

TM_HD GalerkinZ galerkin_layout(const FineGeom& g, int c0, int cb) {
  GalerkinZ z;
  int off = 0;
  for (int p = 0; p < 9; ++p) {
    const int sz = p == 0 ? g.bvol : g.bvol / g.B[(p - 1) >> 1];
    z.regoff[p] = off;
    z.regsz[p] = sz;
    off += sz;
  }
  z.za = off;
  z.c0 = c0;
  z.cb = cb;
  return z;
}

// index of a face site (local coordinates lc) inside the mu-face region:
// lexicographic over the three other directions
TM_D int face_index(const FineGeom& g, const int lc[4], int mu) {
  int r = 0, st = 1;
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    r += lc[nu] * st;
    st *= g.B[nu];
  }
  return r;
}
// inverse: local index (inside the aggregate) of face site r on the face lc_mu = cm
TM_D int face_local(const FineGeom& g, int r, int mu, int cm) {
  int lc[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) {
      lc[nu] = cm;
      continue;
    }
    lc[nu] = r % g.B[nu];
    r /= g.B[nu];
  }
  return ((lc[3] * g.B[2] + lc[2]) * g.B[1] + lc[1]) * g.B[0] + lc[0];
}

TM_D int block_index(const FineGeom& g, const int bc[4]) {
  return ((bc[3] * g.NB[2] + bc[2]) * g.NB[1] + bc[1]) * g.NB[0] + bc[0];
}

// workgroup w of a grid of ceil(n/8)*8*m: the m work items of one
// aggregate share w % 8, i.e. one XCD
TM_D bool xcd_decode(int w, int n, int m, int& agg, int& item) {
  const int x = w & 7, rest = w >> 3;
  item = rest % m;
  agg = (rest / m) * 8 + x;
  return agg < n;
}

template <int MU, typename T>
TM_D void lds_spinor(const cplx<T>* wl, int bv, int sp, int nl, cplx<T>* pn) {
#pragma unroll
  for (int k = 0; k < 12; ++k) pn[k] = (k / 6 == sp) ? wl[(k % 6) * bv + nl] : mk<T>(0, 0);
}

// One direction of k_galerkin_z: the two links at x (U_mu(x) and
// U_mu(x - mu)) serve the aggregate-internal forward and backward hops
// (accumulated into v0, part 0) and the two face hops that leave the
// aggregate through its lower (part 1 + 2 mu) and upper (part 2 + 2 mu) mu
// face, which are written to the receiving aggregate's slot at once.
template <int MU, typename T>
TM_D void galerkin_z_dir(const FineOp<T>& op, const cplx<T>* wl, int sp, long s, int loc, const int c[4],
                         const int yc[4], const cplx<T>* wx, cplx<T>* v0, cplx<T>* Z, const GalerkinZ& zl, int jl,
                         long slot) {
  const FineGeom& g = op.g;
  const int lc = c[MU] % g.B[MU];
  const long sb = fine_neighbour(g, s, c, MU, -1);
  const M3<T> uf = load_link(op.links, MU, s, g.V);
  const M3<T> ub = load_link(op.links, MU, sb, g.V);
  cplx<T> pn[12];
  if (lc < g.B[MU] - 1) {
    lds_spinor<MU>(wl, g.bvol, sp, loc + g.lstride[MU], pn);
    hop_fwd<MU>(uf, pn, v0);
  }
  if (lc > 0) {
    lds_spinor<MU>(wl, g.bvol, sp, loc - g.lstride[MU], pn);
    hop_bwd<MU>(ub, pn, v0);
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    // side 0: lower face, forward hop at x - mu (step +1); side 1: upper face, backward hop at x + mu (step -1)
    if (side == 0 ? lc != 0 : lc != g.B[MU] - 1) continue;
    const int step = side == 0 ? 1 : -1, part = side == 0 ? 1 + 2 * MU : 2 + 2 * MU;
    cplx<T> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = mk<T>(0, 0);
    long ts;
    if (side == 0) {
      ts = sb;
      hop_fwd<MU>(ub, wx, v);
    } else {
      ts = fine_neighbour(g, s, c, MU, +1);
      hop_bwd<MU>(uf, wx, v);
    }
    int rc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) rc[m] = m == MU ? (yc[m] - step + g.NB[m]) % g.NB[m] : yc[m];
    const long recv = block_index(g, rc);
    int tc[4];
    fine_coords(g, ts, tc);
    int tl[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) tl[m] = tc[m] % g.B[m];
    const int r = face_index(g, tl, MU);
    cplx<T>* zo = Z + recv * slot + (long)zl.regoff[part] * 12 * zl.cb + (long)jl * 12 * zl.regsz[part] + r;
#pragma unroll
    for (int k = 0; k < 12; ++k) zo[(long)k * zl.regsz[part]] = v[k];
  }
}

template <typename T, typename S>
__global__ void __launch_bounds__(256) k_galerkin_z(FineOp<T> op, const SP<S>* __restrict__ P, int nv, GalerkinZ zl,
                                                    cplx<T>* __restrict__ Z) {
  __shared__ cplx<T> wl[6 * 256];
  const FineGeom& g = op.g;
  const long V = g.V;
  const int bv = g.bvol;
  int y, jl;
  if (!xcd_decode(blockIdx.x, g.nblocks, zl.cb, y, jl)) return;
  const int cc = zl.c0 + jl, sp = cc / nv, jv = cc - sp * nv;
  const int loc = threadIdx.x;
  const long s = (long)y * bv + loc;
  int c[4];
  fine_coords(g, s, c);
  cplx<T> wx[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const bool in_s = (k < 6) == (sp == 0);
    wx[k] = in_s ? Store<S>::template ld<T>(P + (long)jv * 12 * V + tsite((unsigned)s, 12) + k * FT) : mk<T>(0, 0);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) wl[k * bv + loc] = sp ? wx[6 + k] : wx[k];
  __syncthreads();
  int yc[4];
  {
    int b = y;
    yc[0] = b % g.NB[0]; b /= g.NB[0];
    yc[1] = b % g.NB[1]; b /= g.NB[1];
    yc[2] = b % g.NB[2];
    yc[3] = b / g.NB[2];
  }
  const long slot = (long)12 * zl.cb * zl.za;   // elements per aggregate
  cplx<T> v0[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v0[k] = mk<T>(0, 0);
  clover_block_mv(op.clover, (unsigned)s, V, wx, v0);
  clover_block_mv(op.clover + 36 * V, (unsigned)s, V, wx + 6, v0 + 6);
  // FP64: one direction at a time (the links of all four do not fit in registers)
  galerkin_z_dir<0>(op, wl, sp, s, loc, c, yc, wx, v0, Z, zl, jl, slot);
  if constexpr (sizeof(T) == 8) compiler_fence(v0);
  galerkin_z_dir<1>(op, wl, sp, s, loc, c, yc, wx, v0, Z, zl, jl, slot);
  if constexpr (sizeof(T) == 8) compiler_fence(v0);
  galerkin_z_dir<2>(op, wl, sp, s, loc, c, yc, wx, v0, Z, zl, jl, slot);
  if constexpr (sizeof(T) == 8) compiler_fence(v0);
  galerkin_z_dir<3>(op, wl, sp, s, loc, c, yc, wx, v0, Z, zl, jl, slot);
  cplx<T>* zo = Z + (long)y * slot + (long)jl * 12 * zl.regsz[0] + loc;
#pragma unroll
  for (int k = 0; k < 12; ++k) zo[(long)k * zl.regsz[0]] = v0[k];
}

// D_c[r][part][c0 + j][i] = sum_x sum_{k in chirality of i} conj(P_i(x)_k) Z(x)_{k j}
// thread: column j = t % 16 of the chunk, rows i = t / 16 + 16 a
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_galerkin_proj(FineGeom g, const SP<S>* __restrict__ P, int nv, GalerkinZ zl,
                                                       const cplx<T>* __restrict__ Z, SP<S>* __restrict__ Dc) {
  constexpr int TS = sizeof(T) == 4 ? 8 : 4;   // sites per LDS tile
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* Pt = reinterpret_cast<cplx<T>*>(smem_raw);   // [TS][12][nv]
  cplx<T>* Zt = Pt + TS * 12 * nv;                      // [TS][12][cb]
  int r, part;
  if (!xcd_decode(blockIdx.x, g.nblocks, 9, r, part)) return;
  const long V = g.V;
  const int no = 2 * nv, cb = zl.cb, rs = zl.regsz[part];
  const int t = threadIdx.x, jg = t & 15, ig = t >> 4;
  const int na = (no + 15) / 16;
  int mu = 0, cm = 0;
  if (part > 0) {
    mu = (part - 1) >> 1;
    cm = ((part - 1) & 1) ? 0 : g.B[mu] - 1;   // upper face for the forward neighbour
  }
  const cplx<T>* zr = Z + (long)r * 12 * cb * zl.za + (long)zl.regoff[part] * 12 * cb;
  cplx<T> acc[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) acc[a] = mk<T>(0, 0);
  for (int x0 = 0; x0 < rs; x0 += TS) {
    const int nx = min(TS, rs - x0);
    for (int e = t; e < nx * 12 * nv; e += 256) {
      const int x = e % nx, rem = e / nx, k = rem % 12, iv = rem / 12;
      const int loc = part == 0 ? x0 + x : face_local(g, x0 + x, mu, cm);
      const long site = (long)r * g.bvol + loc;
      Pt[(x * 12 + k) * nv + iv] = Store<S>::template ld<T>(P + (long)iv * 12 * V + tsite((unsigned)site, 12) + k * FT);
    }
    for (int e = t; e < nx * 12 * cb; e += 256) {
      const int x = e % nx, rem = e / nx, k = rem % 12, j = rem / 12;
      Zt[(x * 12 + k) * cb + j] = zr[(long)(j * 12 + k) * rs + x0 + x];
    }
    __syncthreads();
    if (jg < cb) {
#pragma unroll 1
      for (int x = 0; x < nx; ++x) {
        cplx<T> zk[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) zk[k] = Zt[(x * 12 + k) * cb + jg];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const int i = ig + 16 * a;
          if (a < na && i < no) {
            const int sc = i >= nv ? 1 : 0, iv = i - sc * nv;
            const cplx<T>* pr = Pt + (x * 12 + 6 * sc) * nv + iv;
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) cfmac(acc[a], pr[kk * nv], sc ? zk[6 + kk] : zk[kk]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (jg < cb) {
    const int j = zl.c0 + jg;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int i = ig + 16 * a;
      if (a < na && i < no) Store<S>::st(Dc + (((long)r * 9 + part) * no + j) * no + i, acc[a]);
    }
  }
}

// The same projection with the site sum split over the four waves and a
// register block of RPL x 4 outputs per lane: tiles of sites of P (all N_v vectors)
// and Z (the chunk's columns) in LDS; wave w takes sites x = w (mod 4) of
// a tile, lane (rg, cgp) the rows of chirality rg / 8, vectors
// iv = rg % 8 + 8 a (a < RPL), and the columns 4 cgp .. 4 cgp + 3, so each
// LDS value read feeds several products.  The waves' partial sums meet in LDS at the end.
template <typename T> constexpr int gp_ts() { return 16; }   // sites per tile (two workgroups per CU)

template <typename T, typename S, int RPL>
__global__ void __launch_bounds__(256) k_galerkin_proj4(FineGeom g, const SP<S>* __restrict__ P, int nv,
                                                        GalerkinZ zl, const cplx<T>* __restrict__ Z,
                                                        SP<S>* __restrict__ Dc) {
  constexpr int GP_TS = gp_ts<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // site strides padded by one element so that the 32 sites of a tile
  // written by consecutive lanes fall into different LDS banks
  const int PS = 12 * nv + 1, ZS = 12 * zl.cb + 1;
  cplx<T>* Pt = reinterpret_cast<cplx<T>*>(smem_raw);   // [GP_TS][PS]: [x][k][iv]
  cplx<T>* Zt = Pt + GP_TS * PS;                        // [GP_TS][ZS]: [x][k][j]
  int r, part;
  if (!xcd_decode(blockIdx.x, g.nblocks, 9, r, part)) return;
  const long V = g.V;
  const int no = 2 * nv, cb = zl.cb, rs = zl.regsz[part];
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int rg = lane & 15, cgp = lane >> 4, sc = rg >> 3;
  int mu = 0, cm = 0;
  if (part > 0) {
    mu = (part - 1) >> 1;
    cm = ((part - 1) & 1) ? 0 : g.B[mu] - 1;   // upper face for the forward neighbour
  }
  const cplx<T>* zr = Z + (long)r * 12 * cb * zl.za + (long)zl.regoff[part] * 12 * cb;
  cplx<T> acc[RPL][4];   // RPL = ceil(nv / 8) rows per lane
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = mk<T>(0, 0);
  // loads: thread t stages site x = t % GP_TS of the tile, pairs (k, iv) or
  // (k, j) stepping by 256 / GP_TS, so the site index is formed once
  constexpr int XST = 256 / GP_TS;
  const int xt = t % GP_TS, pt0 = t / GP_TS;
  for (int x0 = 0; x0 < rs; x0 += GP_TS) {
    const int nx = min(GP_TS, rs - x0);
    if (xt < nx) {
      const int loc = part == 0 ? x0 + xt : face_local(g, x0 + xt, mu, cm);
      const SP<S>* pb = P + tsite((unsigned)((long)r * g.bvol + loc), 12);
      for (int kv = pt0; kv < 12 * nv; kv += XST) {
        const int k = kv % 12, iv = kv / 12;
        Pt[xt * PS + k * nv + iv] = Store<S>::template ld<T>(pb + (long)iv * 12 * V + k * FT);
      }
      const cplx<T>* zb = zr + x0 + xt;
      for (int kj = pt0; kj < 12 * cb; kj += XST) {
        const int k = kj % 12, j = kj / 12;
        Zt[xt * ZS + k * cb + j] = zb[(long)(j * 12 + k) * rs];
      }
    }
    __syncthreads();
    for (int x = wv; x < nx; x += 4) {
#pragma unroll 2
      for (int kk = 0; kk < 6; ++kk) {
        const int k = 6 * sc + kk;
        cplx<T> pv[RPL], zv[4];
#pragma unroll
        for (int a = 0; a < RPL; ++a) {
          const int iv = (rg & 7) + 8 * a;
          pv[a] = iv < nv ? Pt[x * PS + k * nv + iv] : mk<T>(0, 0);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = 4 * cgp + b;
          zv[b] = j < cb ? Zt[x * ZS + k * cb + j] : mk<T>(0, 0);
        }
#pragma unroll
        for (int a = 0; a < RPL; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) cfmac(acc[a][b], pv[a], zv[b]);
      }
    }
    __syncthreads();
  }
  // partial sums of the four waves: red[w][a][b][lane]
  cplx<T>* red = Pt;
#pragma unroll
  for (int a = 0; a < RPL; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) red[((wv * 4 + a) * 4 + b) * 64 + lane] = acc[a][b];
  __syncthreads();
  for (int e = t; e < RPL * 4 * 64; e += 256) {
    const int ln = e & 63, ab = e >> 6, a = ab >> 2, b = ab & 3;
    const int rg2 = ln & 15, cg2 = ln >> 4, sc2 = rg2 >> 3;
    const int iv = (rg2 & 7) + 8 * a, j = 4 * cg2 + b;
    if (iv < nv && j < cb) {
      cplx<T> sum = red[(a * 4 + b) * 64 + ln];
      for (int w2 = 1; w2 < 4; ++w2) sum += red[((w2 * 4 + a) * 4 + b) * 64 + ln];
      const int i = sc2 * nv + iv;
      Store<S>::st(Dc + (((long)r * 9 + part) * no + zl.c0 + j) * no + i, sum);
    }
  }
}

// The projection on the matrix cores (bf16 P, FP32 Z, N_v <= 32, at most
// 16 columns): per chirality s the block is a (N_v x K) x (K x cb) product
// over K = sites x 6 components,
//   Re = Re P . Re Z + Im P . Im Z,   Im = Re P . Im Z - Im P . Re Z,
// with P exact in bf16 and Z split into two bf16 parts (Z to 2^-18 of its
// size), run as 16x16x32 bf16 MFMA tiles with FP32 accumulation.  Wave w
// owns chirality w / 2 and row tile w % 2 (vectors 16 (w % 2) ..), so the
// waves need no reduction.  Tiles of 16 sites of P (raw bf16 pairs) and Z
// in LDS, loaded as in k_galerkin_proj4.

__global__ void __launch_bounds__(256) k_galerkin_proj_mf(FineGeom g, const bf16pair* __restrict__ P, int nv,
                                                          GalerkinZ zl, const cplx<float>* __restrict__ Z,
                                                          bf16pair* __restrict__ Dc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int PS = 12 * nv + 1, ZS = 12 * zl.cb + 1;
  unsigned* Pt = reinterpret_cast<unsigned*>(smem_raw);                 // [GPM_TS][PS]: [x][k][iv], bf16 pairs
  cplx<float>* Zt = reinterpret_cast<cplx<float>*>(Pt + ((GPM_TS * PS + 1) & ~1));   // [GPM_TS][ZS]: [x][k][j]
  int r, part;
  if (!xcd_decode(blockIdx.x, g.nblocks, 9, r, part)) return;
  const long V = g.V;
  const int no = 2 * nv, cb = zl.cb, rs = zl.regsz[part];
  const int t = threadIdx.x, wv = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  const int sc = wv >> 1, mt = wv & 1;   // chirality and row tile of this wave
  int mu = 0, cm = 0;
  if (part > 0) {
    mu = (part - 1) >> 1;
    cm = ((part - 1) & 1) ? 0 : g.B[mu] - 1;
  }
  const cplx<float>* zr = Z + (long)r * 12 * cb * zl.za + (long)zl.regoff[part] * 12 * cb;
  const unsigned* Pu = reinterpret_cast<const unsigned*>(P);
  mf_f4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  constexpr int XST = 256 / GPM_TS;
  const int xt = t % GPM_TS, pt0 = t / GPM_TS;
  const int iv = 16 * mt + lr;   // this lane's row of A
  for (int x0 = 0; x0 < rs; x0 += GPM_TS) {
    const int nx = min(GPM_TS, rs - x0);
    if (xt < nx) {
      const int loc = part == 0 ? x0 + xt : face_local(g, x0 + xt, mu, cm);
      const unsigned* pb = Pu + tsite((unsigned)((long)r * g.bvol + loc), 12);
      for (int kv = pt0; kv < 12 * nv; kv += XST) {
        const int k = kv % 12, v = kv / 12;
        Pt[xt * PS + k * nv + v] = pb[(long)v * 12 * V + k * FT];
      }
      const cplx<float>* zb = zr + x0 + xt;
      for (int kj = pt0; kj < 12 * cb; kj += XST) {
        const int k = kj % 12, j = kj / 12;
        Zt[xt * ZS + k * cb + j] = zb[(long)(j * 12 + k) * rs];
      }
    }
    __syncthreads();
    // K steps of 16 over (site, component of chirality sc): kk = x * 6 + k
    const int nk = nx * 6;
    for (int k0 = 0; k0 < nk; k0 += 16) {
      mf_s4 ar, ai;
      cplx<float> zv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = k0 + 4 * lk + e;
        const int x = kk / 6, kc = 6 * sc + kk % 6;
        unsigned u = 0u;
        cplx<float> z = mk<float>(0, 0);
        if (kk < nk) {
          if (iv < nv) u = Pt[x * PS + kc * nv + iv];
          if (lr < cb) z = Zt[x * ZS + kc * cb + lr];
        }
        ar[e] = (short)(u & 0xffffu);
        ai[e] = (short)(u >> 16);
        zv[e] = z;
      }
      const MfSplit bb = mf_split(zv);
      mf_cmac_conj(ar, ai, bb, accr, acci);
    }
    __syncthreads();
  }
  // C tile: lane l holds rows 4 (l / 16) + v (vector 16 mt + ...), column j = l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int ivo = 16 * mt + 4 * lk + v, j = lr;
    if (ivo < nv && j < cb) {
      const int i = sc * nv + ivo;
      Store<__hip_bfloat16>::st(Dc + (((long)r * 9 + part) * no + zl.c0 + j) * no + i, mk(accr[v], acci[v]));
    }
  }
}

size_t galerkin_ws_per_column(const FineGeom& g) {
  const GalerkinZ z = galerkin_layout(g, 0, 1);
  return (size_t)g.nblocks * 12 * z.za;
}

// columns per chunk for a Z workspace of ws_elems complex values
static int galerkin_chunk(const FineGeom& g, int nv, size_t ws_elems) {
  const size_t per_col = galerkin_ws_per_column(g);
  return (int)std::max<size_t>(1, std::min<size_t>({(size_t)16, (size_t)(2 * nv), ws_elems / per_col}));
}

template <typename T, typename S>
void launch_galerkin_fine(const FineOp<T>& op, const SP<S>* P, int nv, SP<S>* Dc, cplx<T>* zws, size_t zws_elems,
                          hipStream_t st) {
  const FineGeom& g = op.g;
  const int no = 2 * nv;
  if (zws_elems < galerkin_ws_per_column(g)) throw TmError{TMAMG_EINVAL, "Galerkin workspace too small"};
  const int cb = galerkin_chunk(g, nv, zws_elems);
  const int n8 = (g.nblocks + 7) / 8 * 8;
  constexpr int TS = sizeof(T) == 4 ? 8 : 4;
  const size_t lds = (size_t)TS * 12 * (nv + cb) * sizeof(cplx<T>);
  // the register-blocked projection: up to 32 vectors and 16 columns
  const size_t lds4 = (size_t)gp_ts<T>() * (12 * (nv + cb) + 2) * sizeof(cplx<T>);
  // the wave partials (4 waves x RPL x 4 x 64 values) reuse the P and Z tiles
  const int rpl = nv <= 24 ? 3 : 4;
  const bool use4 = nv <= 32 && cb <= 16 && lds4 <= 150 * 1024 &&
                    (size_t)gp_ts<T>() * (12 * (nv + cb) + 2) >= (size_t)rpl * 1024;
  if (use4 && lds4 > 64 * 1024) {
    static bool attr = false;
    if (!attr) {
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_galerkin_proj4<T, S, 3>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_galerkin_proj4<T, S, 4>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
      attr = true;
    }
  }
  for (int c0 = 0; c0 < no; c0 += cb) {
    const GalerkinZ zl = galerkin_layout(g, c0, std::min(cb, no - c0));
    hipLaunchKernelGGL((k_galerkin_z<T, S>), dim3((unsigned)(n8 * zl.cb)), dim3(g.bvol), 0, st, op, P, nv, zl, zws);
    if constexpr (std::is_same<T, float>::value && std::is_same<S, __hip_bfloat16>::value) {
      if (nv <= 32 && zl.cb <= 16) {
        const size_t ldsm = ((size_t)GPM_TS * (12 * nv + 1) + 1) / 2 * 2 * 4 + (size_t)GPM_TS * (12 * zl.cb + 1) * 8;
        hipLaunchKernelGGL(k_galerkin_proj_mf, dim3((unsigned)(n8 * 9)), dim3(256), ldsm, st, g, P, nv, zl, zws, Dc);
        continue;
      }
    }
    if (use4 && rpl == 3)
      hipLaunchKernelGGL((k_galerkin_proj4<T, S, 3>), dim3((unsigned)(n8 * 9)), dim3(256), lds4, st, g, P, nv, zl,
                         zws, Dc);
    else if (use4)
      hipLaunchKernelGGL((k_galerkin_proj4<T, S, 4>), dim3((unsigned)(n8 * 9)), dim3(256), lds4, st, g, P, nv, zl,
                         zws, Dc);
    else
      hipLaunchKernelGGL((k_galerkin_proj<T, S>), dim3((unsigned)(n8 * 9)), dim3(256), lds, st, g, P, nv, zl, zws,
                         Dc);
  }
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
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x) {
    unsigned long long h1 = mix64(seed * 0x632BE59BD9B4E019ULL + 2 * (unsigned long long)k);
    unsigned long long h2 = mix64(h1 ^ (2 * (unsigned long long)k + 1));
    double u1 = ((double)(h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((double)(h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double rad = sqrt(-log(u1));
    double ph = 6.283185307179586 * u2;
    out[k] = mk<T>((T)(rad * cos(ph)), (T)(rad * sin(ph)));
  }
}
template <typename T>
void launch_random(cplx<T>* out, long count, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(k_random<T>, dim3(grid1d(count)), dim3(256), 0, st, out, count, seed);
}

template <typename S>
__global__ void k_store_to64(const SP<S>* in, cplx<double>* out, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x)
    out[k] = Store<S>::template ld<double>(in + k);
}
template <typename S>
__global__ void k_store_from64(const cplx<double>* in, SP<S>* out, long count) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < count; k += (long)gridDim.x * blockDim.x)
    Store<S>::st(out + k, in[k]);
}
template <typename S>
void launch_store_to64(const SP<S>* in, cplx<double>* out, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_store_to64<S>, dim3(grid1d(count)), dim3(256), 0, st, in, out, count);
}
template <typename S>
void launch_store_from64(const cplx<double>* in, SP<S>* out, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_store_from64<S>, dim3(grid1d(count)), dim3(256), 0, st, in, out, count);
}

#define INST_TS(T, S)                                                                                            \
  template void launch_restrict_fine<T, S>(const FineGeom&, const SP<S>*, int, const cplx<T>*, cplx<T>*, int,    \
                                           hipStream_t);                                                         \
  template void launch_prolong_fine<T, S>(const FineGeom&, const SP<S>*, int, const cplx<T>*, cplx<T>*, int,     \
                                          hipStream_t);                                                          \
  template void launch_gs_fine<T, S>(const FineGeom&, const cplx<T>*, int, cplx<double>*, SP<S>*, hipStream_t);  \
  template void launch_galerkin_fine<T, S>(const FineOp<T>&, const SP<S>*, int, SP<S>*, cplx<T>*, size_t,  \
                                           hipStream_t);
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
