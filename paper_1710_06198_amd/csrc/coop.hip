// Coarse-level SAP and the coarsest-level GMRES, organised around one
// coarse site per workgroup.
//
// Coarse lattices are small (a few hundred to a few thousand sites), so a
// thread per matrix row is latency-bound.  Here a 256-thread workgroup
// stages the nine input vectors a site needs in LDS and forms the D rows of
// D_c with every thread owning four consecutive rows and a slice of the
// 9*D-term sum (one 4-wide vector load per term), followed by an LDS
// reduction over the slices.
//
// Global synchronisation is priced by what it costs on a chip of 8 XCDs: a
// grid-wide barrier over a thousand workgroups costs tens of microseconds,
// a kernel boundary about two and a half.  The SAP smoother therefore uses
// plain launches, one per minimal-residual step, with the update of step k
// folded into the staging of step k+1.  The coarsest GMRES runs as one
// persistent launch on at most a few dozen workgroups that synchronise
// through a counter barrier; each workgroup reduces the per-workgroup
// partial sums itself, in a fixed order, so all of them hold identical
// Gram-Schmidt coefficients without a separate reduction phase.
#include <type_traits>

#include "kernels.h"
#include "mfma.h"
#include "solver.h"

template <typename S> using SP = typename Store<S>::pair;

struct CBlk {
  int B[4], NB[4], nbs;
};

TM_D void cblk_site(const CBlk& cb, int blk, int sl, C4& c, C4& lc) {
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
// in-block neighbour (local index) or -1 when the hop leaves the block
TM_D int cblk_nbr(const CBlk& cb, C4 lc, int mu, int step) {
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
TM_D int hop_mu(int b) { return (b - 1) >> 1; }
TM_D int hop_step(int b) { return ((b - 1) & 1) ? -1 : 1; }

// Source site of each of the nine blocks of site y (the site itself, then
// its neighbours), formed once per workgroup in LDS rather than per staged
// element; ends with a barrier.  The in-block variant gives -1 where the
// hop leaves the SAP block.
TM_D void stage_sources(const CoarseGeom& g, long y, const C4& c, long* src9) {
  if (threadIdx.x < 9) {
    const int b = threadIdx.x;
    src9[b] = b == 0 ? y : cc_nbr(g, c, hop_mu(b), hop_step(b));
  }
  __syncthreads();
}
TM_D void stage_block_sources(const CoarseGeom& g, const CBlk& cb, int blk, long y, const C4& lc, long* src9) {
  if (threadIdx.x < 9) {
    const int b = threadIdx.x;
    long v = y;
    if (b != 0) {
      const int nl = cblk_nbr(cb, lc, hop_mu(b), hop_step(b));
      if (nl < 0) {
        v = -1;
      } else {
        C4 cn, lcn;
        cblk_site(cb, blk, nl, cn, lcn);
        v = cc_index(g, cn);
      }
    }
    src9[b] = v;
  }
  __syncthreads();
}

// Partial products of one site's D rows for NR right-hand sides:
// red[q][ks][i] summed over ks gives
//   sum_{b in mask} sum_j Dm[b][j][i] vst[q][b*D + j].
// Every thread owns four consecutive rows and a slice of the 9*D-term sum;
// one 4-wide load of D_c serves all NR vectors.  Ends with a workgroup
// barrier.
template <int D> struct SiteMV {
  static constexpr int RG = D / 4;      // row groups of 4 rows
  static constexpr int KS = 256 / RG;   // slices of the 9*D-term sum
};
template <typename T, typename S, int D, int NR = 1>
TM_D void site_mv(const SP<S>* __restrict__ Dm, const cplx<T>* vst, unsigned mask, cplx<T>* red) {
  constexpr int RG = SiteMV<D>::RG, KS = SiteMV<D>::KS, K = 9 * D;
  const int t = threadIdx.x, rg = t % RG, ks = t / RG;
  if (ks < KS) {
    cplx<T> a[NR][4];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) a[q][i] = mk<T>(0, 0);
#pragma unroll 4
    for (int k = ks; k < K; k += KS) {
      const int b = k / D;
      if (!((mask >> b) & 1u)) continue;
      const Quad<S> qd = *reinterpret_cast<const Quad<S>*>(Dm + (size_t)k * D + 4 * rg);
      cplx<T> m4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) m4[i] = Store<S>::template cvt<T>(qd.e[i]);
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const cplx<T> v = vst[q * K + k];
#pragma unroll
        for (int i = 0; i < 4; ++i) cfma(a[q][i], m4[i], v);
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      cplx<T>* o = red + (q * KS + ks) * D + 4 * rg;
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = a[q][i];
    }
  }
  __syncthreads();
}
template <typename T, int D>
TM_D cplx<T> site_mv_row(const cplx<T>* red, int i) {
  cplx<T> s = mk<T>(0, 0);
  for (int ks = 0; ks < SiteMV<D>::KS; ++ks) s += red[ks * D + i];
  return s;
}

// ------------------------------------------------------------------ batched site rows on the matrix cores
// With 16 right-hand sides and a bf16 D_c the product of site_mv,
//   out[q][i] = sum_{b in mask} sum_j D_b(i, j) v[q][b D + j],
// is a complex (D x 9D) x (9D x 16) matrix product.  It runs as real
// bf16 MFMA products (16x16x32, mf_cmac) with FP32 accumulation:
//   Re out = Re D Re v - Im D Im v,   Im out = Re D Im v + Im D Re v.
// The D_c entries are exact in bf16.  Each FP32 vector entry is split as
// v = v_hi + v_lo, v_hi = bf16(v), v_lo = bf16(v - v_hi), which keeps v to
// 2^-18 of its size, so a 16x16 tile takes 4 products per 16 terms of the
// sum.  Wave w takes the blocks b = w (mod 4) for all row tiles; the four
// partial sums are left in the slots of blocks 1..4 of vst (the own-site
// slot, block 0, keeps the input) and summed by the reader.
constexpr int MF_NR = 16;   // right-hand sides per workgroup on the matrix cores

template <typename T, typename S, int D> constexpr bool mf_ok() {
  return std::is_same<T, float>::value && std::is_same<S, __hip_bfloat16>::value && D % 16 == 0;
}

// vst: [16][stride] staged inputs, block b's D values at slot[b] * D (slot
// == nullptr: slot b); on return (after a barrier) the partial sums of wave
// w are at vst[q * stride + (1 + w) D + i] (slots 1..4 must exist)
// The D_c fragments a wave needs first, loaded ahead of the staging of the
// inputs so that their latency overlaps it: wave w takes the blocks
// b = w (mod 4) of the mask, 4 bits each in `blocks`.
template <int D>
struct MfPre {
  static constexpr int MT = D / 16, KS = D / 16;
  unsigned an[KS][MT][4];
  int blocks, nb;
};
template <int D>
TM_D void mf_load_block(const unsigned* __restrict__ Du, int b, unsigned (&an)[D / 16][D / 16][4]) {
  constexpr int MT = D / 16, KS = D / 16;
  const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  const unsigned* dp = Du + (size_t)(b * D + 4 * lk) * D + lr;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int e = 0; e < 4; ++e) an[ks][mt][e] = dp[(16 * ks + e) * D + 16 * mt];
}
template <int D>
TM_D void mf_prefetch(const bf16pair* __restrict__ Dm, unsigned mask, MfPre<D>& pre) {
  const int w = threadIdx.x >> 6;
  pre.blocks = 0;
  pre.nb = 0;
  for (int b = w; b < 9; b += 4)
    if ((mask >> b) & 1u) pre.blocks |= b << (4 * pre.nb++);
  if (pre.nb > 0) mf_load_block<D>(reinterpret_cast<const unsigned*>(Dm), pre.blocks & 15, pre.an);
}

// vst: [16][stride] staged inputs, block b's D values at slot[b] * D (slot
// == nullptr: slot b); on return (after a barrier) the partial sums of wave
// w are at vst[q * stride + (1 + w) D + i] (slots 1..4 must exist).  pre
// holds the wave's first D_c fragments (mf_prefetch).
template <int D>
TM_D void site_mv_mfma_pre(const bf16pair* __restrict__ Dm, cplx<float>* vst, MfPre<D>& pre, int stride = 9 * D,
                           const int* slot = nullptr) {
  constexpr int MT = D / 16, KS = D / 16;
  const int K9 = stride;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  const unsigned* __restrict__ Du = reinterpret_cast<const unsigned*>(Dm);
  mf_f4 accr[MT], acci[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) accr[mt] = acci[mt] = mf_f4{0.f, 0.f, 0.f, 0.f};
  // all D_c fragments of the next block are loaded while the current block
  // runs on the matrix cores
  for (int ib = 0; ib < pre.nb; ++ib) {
    unsigned ac[KS][MT][4];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) ac[ks][mt][e] = pre.an[ks][mt][e];
    if (ib + 1 < pre.nb) mf_load_block<D>(Du, (pre.blocks >> (4 * (ib + 1))) & 15, pre.an);
    const int b = (pre.blocks >> (4 * ib)) & 15;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int j0 = 16 * ks + 4 * lk;
      cplx<float> v4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v4[e] = vst[lr * K9 + (slot ? slot[b] : b) * D + j0 + e];
      const MfSplit bb = mf_split(v4);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        mf_s4 ar, ai;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ar[e] = (short)(ac[ks][mt][e] & 0xffffu);
          ai[e] = (short)(ac[ks][mt][e] >> 16);
        }
        mf_cmac(ar, ai, bb, accr[mt], acci[mt]);
      }
    }
  }
  __syncthreads();   // every wave has read the neighbour slots
  // C tile layout: lane l holds rows 4 (l / 16) + v of the tile, column l % 16
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) vst[lr * K9 + (1 + w) * D + 16 * mt + 4 * lk + v] = mk(accr[mt][v], acci[mt][v]);
  __syncthreads();
}
template <int D>
TM_D void site_mv_mfma(const bf16pair* __restrict__ Dm, cplx<float>* vst, unsigned mask, int stride = 9 * D,
                       const int* slot = nullptr) {
  MfPre<D> pre;
  mf_prefetch<D>(Dm, mask, pre);
  site_mv_mfma_pre<D>(Dm, vst, pre, stride, slot);
}
template <int D>
TM_D cplx<float> site_mv_mfma_row(const cplx<float>* vst, int q, int i, int stride = 9 * D) {
  const cplx<float>* p = vst + q * stride + D + i;
  return (p[0] + p[D]) + (p[2 * D] + p[3 * D]);
}

// D_c(mu_r) for 16 right-hand sides per workgroup (one coarse site) on the
// matrix cores; vst is dynamic LDS of 16 * 9 D complex values
template <int D>
__global__ void __launch_bounds__(256) k_coarse_apply_mf(CoarseGeom g, const bf16pair* __restrict__ Dc,
                                                         const cplx<float>* __restrict__ in,
                                                         cplx<float>* __restrict__ out, int nrhs,
                                                         const double* __restrict__ mu_dev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<float>* vst = reinterpret_cast<cplx<float>*>(smem_raw);
  const long y = blockIdx.x;
  const int r0 = blockIdx.y * MF_NR;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  const C4 c = cc_coords(g, y);
  MfPre<D> pre;   // first D_c fragments ahead of the staging
  mf_prefetch<D>(Dc + y * 9L * D * D, 0x1FFu, pre);
  __shared__ long src9[9];
  stage_sources(g, y, c, src9);
  for (int k2 = t; k2 < MF_NR * 9 * D / 2; k2 += 256) {   // two complex values per 16-byte access
    const int k = 2 * k2, q = k / (9 * D), kk = k - q * 9 * D, b = kk / D, j = kk - b * D;
    const long src = src9[b];
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + q < nrhs) v = *reinterpret_cast<const float4*>(in + (r0 + q) * VD + src * D + j);
    *reinterpret_cast<float4*>(vst + k) = v;
  }
  __syncthreads();
  site_mv_mfma_pre<D>(Dc + y * 9L * D * D, vst, pre);
  for (int e = t; e < MF_NR * D; e += 256) {
    const int q = e / D, i = e - q * D, r = r0 + q;
    if (r >= nrhs) continue;
    const float mu = (float)mu_dev[r];
    cplx<float> acc = site_mv_mfma_row<D>(vst, q, i);
    acc += (i < D / 2 ? mu : -mu) * times_i(vst[q * 9 * D + i]);
    out[r * VD + y * D + i] = acc;
  }
}

template <int D>
static void coarse_apply_mf(const CoarseGeom& g, const bf16pair* Dc, const cplx<float>* in, cplx<float>* out,
                            int nrhs, const double* mu_dev, hipStream_t st) {
  const size_t lds = (size_t)MF_NR * 9 * D * sizeof(cplx<float>);
  static bool attr = false;
  if (!attr && lds > 64 * 1024) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_apply_mf<D>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  hipLaunchKernelGGL((k_coarse_apply_mf<D>), dim3((unsigned)g.V, (nrhs + MF_NR - 1) / MF_NR), dim3(256), lds, st, g,
                     Dc, in, out, nrhs, mu_dev);
}

// ------------------------------------------------------------------ coarse operator, one site per workgroup
// D_c(mu_r) for NR right-hand sides per workgroup (one coarse site), with
// the slice mapping of site_mv: 16-byte D_c loads, many in flight per
// thread, shared by the NR vectors.
template <typename T, typename S, int D, int NR>
__global__ void __launch_bounds__(256) k_coarse_apply_site(CoarseGeom g, const SP<S>* __restrict__ Dc,
                                                           const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                           int nrhs, const double* __restrict__ mu_dev) {
  __shared__ cplx<T> vst[NR * 9 * D];
  __shared__ cplx<T> red[NR * SiteMV<D>::KS * D];
  const long y = blockIdx.x;
  const int r0 = blockIdx.y * NR;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  const C4 c = cc_coords(g, y);
  __shared__ long src9[9];
  stage_sources(g, y, c, src9);
  for (int k = t; k < NR * 9 * D; k += 256) {
    const int q = k / (9 * D), kk = k - q * 9 * D, b = kk / D, j = kk - b * D;
    const long src = src9[b];
    vst[k] = r0 + q < nrhs ? in[(r0 + q) * VD + src * D + j] : mk<T>(0, 0);
  }
  __syncthreads();
  site_mv<T, S, D, NR>(Dc + y * 9L * D * D, vst, 0x1FFu, red);
  for (int e = t; e < NR * D; e += 256) {
    const int q = e / D, i = e - q * D, r = r0 + q;
    if (r >= nrhs) continue;
    const T mu = (T)mu_dev[r];
    cplx<T> acc = site_mv_row<T, D>(red + q * SiteMV<D>::KS * D, i);
    acc += (i < D / 2 ? mu : -mu) * times_i(vst[q * 9 * D + i]);
    out[r * VD + y * D + i] = acc;
  }
}

template <typename T, typename S, int D>
static void coarse_apply_site(const CoarseGeom& g, const SP<S>* Dc, const cplx<T>* in, cplx<T>* out, int nrhs,
                              const double* mu_dev, hipStream_t st) {
  if constexpr (mf_ok<T, S, D>()) {
    const int tv = tune_get(TUNE_COARSE_APPLY, D, g.V, nrhs);
    if (tv >= 0 ? tv == 1 : nrhs >= 8) {
      coarse_apply_mf<D>(g, Dc, in, out, nrhs, mu_dev, st);
      tune_used(TUNE_COARSE_APPLY, 1);
      return;
    }
  }
  tune_used(TUNE_COARSE_APPLY, 0);
  if (nrhs >= 4)
    hipLaunchKernelGGL((k_coarse_apply_site<T, S, D, 4>), dim3((unsigned)g.V, (nrhs + 3) / 4), dim3(256), 0, st, g,
                       Dc, in, out, nrhs, mu_dev);
  else
    hipLaunchKernelGGL((k_coarse_apply_site<T, S, D, 1>), dim3((unsigned)g.V, nrhs), dim3(256), 0, st, g, Dc, in,
                       out, nrhs, mu_dev);
}

template <typename T, typename S>
bool launch_coarse_apply_site(const CoarseGeom& g, int d, const SP<S>* Dc, const cplx<T>* in, cplx<T>* out,
                              int nrhs, const double* mu_dev, hipStream_t st) {
  switch (d) {
    case 24: coarse_apply_site<T, S, 24>(g, Dc, in, out, nrhs, mu_dev, st); return true;
    case 32: coarse_apply_site<T, S, 32>(g, Dc, in, out, nrhs, mu_dev, st); return true;
    case 48: coarse_apply_site<T, S, 48>(g, Dc, in, out, nrhs, mu_dev, st); return true;
    case 64: coarse_apply_site<T, S, 64>(g, Dc, in, out, nrhs, mu_dev, st); return true;
    default: return false;
  }
}

// ------------------------------------------------------------------ SAP with fused MR steps
struct SapArgs {
  CoarseGeom g;
  CBlk cb;
  const int* bl;   // blocks of the colour being solved
  int nrhs;
};

// unit u -> (block of the colour, site of the block, group of NR
// right-hand sides r0 .. r0 + NR - 1)
template <int NR>
TM_D void sap_unit(const SapArgs& a, int u, int& bi, int& sl, int& r0) {
  const int ng = (a.nrhs + NR - 1) / NR;
  r0 = (u % ng) * NR;
  const int tt = u / ng;
  sl = tt % a.cb.nbs;
  bi = tt / a.cb.nbs;
}

// MR step sizes of a block for NR right-hand sides: alpha = (q, rho) /
// (q, q), summed over the block's sites in a fixed order from per-site
// partials (q.q, q^H rho).  Wave q handles right-hand side r0 + q.
template <typename T, int NR>
TM_D void block_alpha(const double* __restrict__ part, int bi, int nbs, int nrhs, int r0, cplx<T>* alpha_s) {
  const int t = threadIdx.x, q = t >> 6, lane = t & 63;
  for (int qq = q; qq < NR; qq += 4) {
    const int r = r0 + qq;
    double sq = 0, sre = 0, sim = 0;
    if (r < nrhs)
      for (int p = lane; p < nbs; p += 64) {
        const long o = 3L * (((long)bi * nbs + p) * nrhs + r);
        sq += part[o];
        sre += part[o + 1];
        sim += part[o + 2];
      }
    sq = wave_sum(sq);
    sre = wave_sum(sre);
    sim = wave_sum(sim);
    if (lane == 0) alpha_s[qq] = sq > 0 ? mk<T>((T)(sre / sq), (T)(sim / sq)) : mk<T>(0, 0);
  }
  __syncthreads();
}

// rho = eta - D_c(mu) z on the sites of the colour's blocks
template <typename T, typename S, int D, int NR>
__global__ void __launch_bounds__(256) k_sap1_resid(SapArgs a, const SP<S>* __restrict__ Dc,
                                                    const cplx<T>* __restrict__ eta, const cplx<T>* __restrict__ z,
                                                    cplx<T>* __restrict__ rho, const double* __restrict__ mu_dev) {
  __shared__ cplx<T> vst[NR * 9 * D];
  __shared__ cplx<T> red[NR * SiteMV<D>::KS * D];
  const CoarseGeom& g = a.g;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  int bi, sl, r0;
  sap_unit<NR>(a, blockIdx.x, bi, sl, r0);
  C4 c, lc;
  cblk_site(a.cb, a.bl[bi], sl, c, lc);
  const long y = cc_index(g, c);
  __shared__ long src9[9];
  stage_sources(g, y, c, src9);
  for (int k = t; k < NR * 9 * D; k += 256) {
    const int q = k / (9 * D), kk = k - q * 9 * D, b = kk / D, j = kk - b * D;
    const long src = src9[b];
    vst[k] = r0 + q < a.nrhs ? z[(r0 + q) * VD + src * D + j] : mk<T>(0, 0);
  }
  __syncthreads();
  site_mv<T, S, D, NR>(Dc + y * 9L * D * D, vst, 0x1FFu, red);
  for (int e = t; e < NR * D; e += 256) {
    const int q = e / D, i = e - q * D, r = r0 + q;
    if (r >= a.nrhs) continue;
    const T mu = (T)mu_dev[r];
    cplx<T> acc = site_mv_row<T, D>(red + q * SiteMV<D>::KS * D, i);
    acc += (i < D / 2 ? mu : -mu) * times_i(vst[q * 9 * D + i]);
    rho[r * VD + y * D + i] = eta[r * VD + y * D + i] - acc;
  }
}

// One MR step on every block of the colour.  With first == 0 the previous
// step is completed on the fly: alpha_prev from part_in, rho = rho_in -
// alpha_prev q_in for the staged in-block neighbours, z += alpha_prev
// rho_in on the own site.  Then q = D_B rho, written with rho and the
// per-site partials of the next alpha.
template <typename T, typename S, int D, int NR>
__global__ void __launch_bounds__(256) k_sap1_mr(SapArgs a, const SP<S>* __restrict__ Dc, cplx<T>* __restrict__ z,
                                                 const cplx<T>* __restrict__ rho_in, const cplx<T>* __restrict__ q_in,
                                                 const double* __restrict__ part_in, cplx<T>* __restrict__ rho_out,
                                                 cplx<T>* __restrict__ q_out, double* __restrict__ part_out,
                                                 const double* __restrict__ mu_dev, int first) {
  __shared__ cplx<T> vst[NR * 9 * D];
  __shared__ cplx<T> red[NR * SiteMV<D>::KS * D];
  __shared__ cplx<T> alpha_s[NR];
  const CoarseGeom& g = a.g;
  const CBlk& cb = a.cb;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  int bi, sl, r0;
  sap_unit<NR>(a, blockIdx.x, bi, sl, r0);
  const int blk = a.bl[bi];
  C4 c, lc;
  cblk_site(cb, blk, sl, c, lc);
  const long y = cc_index(g, c);
  if (!first) block_alpha<T, NR>(part_in, bi, cb.nbs, a.nrhs, r0, alpha_s);
  __shared__ long src9[9];
  stage_block_sources(g, cb, blk, y, lc, src9);
  unsigned mask = 0u;
  for (int b = 0; b < 9; ++b)
    if (src9[b] >= 0) mask |= 1u << b;
  for (int k = t; k < NR * 9 * D; k += 256) {
    const int q = k / (9 * D), kk = k - q * 9 * D, b = kk / D, j = kk - b * D, r = r0 + q;
    cplx<T> v = mk<T>(0, 0);
    const long src = src9[b];
    if (src >= 0 && r < a.nrhs) {
      v = rho_in[r * VD + src * D + j];
      if (!first) {
        const cplx<T> al = alpha_s[q];
        const cplx<T> qv = q_in[r * VD + src * D + j];
        v.re -= al.re * qv.re - al.im * qv.im;
        v.im -= al.re * qv.im + al.im * qv.re;
      }
    }
    vst[k] = v;
  }
  __syncthreads();
  site_mv<T, S, D, NR>(Dc + y * 9L * D * D, vst, mask, red);
  // wave q: right-hand side r0 + q (and q + 4, ...), lanes over rows
  const int wq = t >> 6, lane = t & 63;
  for (int q = wq; q < NR; q += 4) {
    const int r = r0 + q;
    if (r >= a.nrhs) continue;   // uniform across the wave
    T qq = 0, qre = 0, qim = 0;
    if (lane < D) {
      const T mu = (T)mu_dev[r];
      const cplx<T> rho = vst[q * 9 * D + lane];
      cplx<T> acc = site_mv_row<T, D>(red + q * SiteMV<D>::KS * D, lane);
      acc += (lane < D / 2 ? mu : -mu) * times_i(rho);
      const long o = r * VD + y * D + lane;
      q_out[o] = acc;
      rho_out[o] = rho;
      if (!first) cfma(z[o], alpha_s[q], rho_in[o]);
      qq = norm2(acc);
      const cplx<T> tq = cmulc(acc, rho);
      qre = tq.re;
      qim = tq.im;
    }
    qq = wave_sum(qq);
    qre = wave_sum(qre);
    qim = wave_sum(qim);
    if (lane == 0) {
      const long u = ((long)bi * cb.nbs + sl) * a.nrhs + r;
      part_out[3 * u] = qq;
      part_out[3 * u + 1] = qre;
      part_out[3 * u + 2] = qim;
    }
  }
}

// completes the last MR step: z += alpha rho
template <typename T, int D, int NR>
__global__ void __launch_bounds__(256) k_sap1_fin(SapArgs a, cplx<T>* __restrict__ z,
                                                  const cplx<T>* __restrict__ rho_in,
                                                  const double* __restrict__ part_in) {
  __shared__ cplx<T> alpha_s[NR];
  const CoarseGeom& g = a.g;
  int bi, sl, r0;
  sap_unit<NR>(a, blockIdx.x, bi, sl, r0);
  block_alpha<T, NR>(part_in, bi, a.cb.nbs, a.nrhs, r0, alpha_s);
  C4 c, lc;
  cblk_site(a.cb, a.bl[bi], sl, c, lc);
  const long y = cc_index(g, c);
  for (int e = threadIdx.x; e < NR * D; e += blockDim.x) {
    const int q = e / D, i = e - q * D, r = r0 + q;
    if (r >= a.nrhs) continue;
    const long o = r * g.V * D + y * D + i;
    cfma(z[o], alpha_s[q], rho_in[o]);
  }
}

// The residual and MR steps for 16 right-hand sides per workgroup on the
// matrix cores (bf16 D_c, FP32 vectors); same data flow as k_sap1_resid
// and k_sap1_mr, vst in dynamic LDS.
// MINB: workgroups per CU the register allocation aims for (4 helps on
// large coarse lattices, where more resident sites hide the D_c loads).
template <int D, int MINB>
__global__ void __launch_bounds__(256, MINB) k_sap1_resid_mf(SapArgs a, const bf16pair* __restrict__ Dc,
                                                       const cplx<float>* __restrict__ eta,
                                                       const cplx<float>* __restrict__ z,
                                                       cplx<float>* __restrict__ rho,
                                                       const double* __restrict__ mu_dev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<float>* vst = reinterpret_cast<cplx<float>*>(smem_raw);
  const CoarseGeom& g = a.g;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  int bi, sl, r0;
  sap_unit<MF_NR>(a, blockIdx.x, bi, sl, r0);
  C4 c, lc;
  cblk_site(a.cb, a.bl[bi], sl, c, lc);
  const long y = cc_index(g, c);
  MfPre<D> pre;   // first D_c fragments ahead of the staging
  mf_prefetch<D>(Dc + y * 9L * D * D, 0x1FFu, pre);
  __shared__ long src9[9];
  stage_sources(g, y, c, src9);
  for (int k2 = t; k2 < MF_NR * 9 * D / 2; k2 += 256) {   // two complex values per 16-byte access
    const int k = 2 * k2, q = k / (9 * D), kk = k - q * 9 * D, b = kk / D, j = kk - b * D;
    const long src = src9[b];
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + q < a.nrhs) v = *reinterpret_cast<const float4*>(z + (r0 + q) * VD + src * D + j);
    *reinterpret_cast<float4*>(vst + k) = v;
  }
  __syncthreads();
  site_mv_mfma_pre<D>(Dc + y * 9L * D * D, vst, pre);
  for (int e = t; e < MF_NR * D; e += 256) {
    const int q = e / D, i = e - q * D, r = r0 + q;
    if (r >= a.nrhs) continue;
    const float mu = (float)mu_dev[r];
    cplx<float> acc = site_mv_mfma_row<D>(vst, q, i);
    acc += (i < D / 2 ? mu : -mu) * times_i(vst[q * 9 * D + i]);
    rho[r * VD + y * D + i] = eta[r * VD + y * D + i] - acc;
  }
}

template <int D, int MINB>
__global__ void __launch_bounds__(256, MINB) k_sap1_mr_mf(SapArgs a, const bf16pair* __restrict__ Dc,
                                                    cplx<float>* __restrict__ z,
                                                    const cplx<float>* __restrict__ rho_in,
                                                    const cplx<float>* __restrict__ q_in,
                                                    const double* __restrict__ part_in,
                                                    cplx<float>* __restrict__ rho_out, cplx<float>* __restrict__ q_out,
                                                    double* __restrict__ part_out, const double* __restrict__ mu_dev,
                                                    int first, int nslot) {
  // only the blocks inside the SAP block are staged: block b in slot
  // slot9[b]; nslot (at least 5, for the partial sums) bounds the count
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<float>* vst = reinterpret_cast<cplx<float>*>(smem_raw);
  __shared__ cplx<float> alpha_s[MF_NR];
  __shared__ int slot9[9], bslot[9];
  const CoarseGeom& g = a.g;
  const CBlk& cb = a.cb;
  const long VD = g.V * D;
  const int t = threadIdx.x;
  int bi, sl, r0;
  sap_unit<MF_NR>(a, blockIdx.x, bi, sl, r0);
  const int blk = a.bl[bi];
  C4 c, lc;
  cblk_site(cb, blk, sl, c, lc);
  const long y = cc_index(g, c);
  // the blocks inside the SAP block, from the local coordinates (the same
  // test as stage_block_sources); the first D_c fragments are requested
  // before anything else so that their latency overlaps the staging
  unsigned mask = 1u;
  for (int b = 1; b < 9; ++b)
    if (cblk_nbr(cb, lc, hop_mu(b), hop_step(b)) >= 0) mask |= 1u << b;
  MfPre<D> pre;
  mf_prefetch<D>(Dc + y * 9L * D * D, mask, pre);
  if (!first) block_alpha<float, MF_NR>(part_in, bi, cb.nbs, a.nrhs, r0, alpha_s);
  __shared__ long src9[9];
  stage_block_sources(g, cb, blk, y, lc, src9);
  if (t == 0) {
    int ns = 0;
    for (int b = 0; b < 9; ++b) {
      slot9[b] = ((mask >> b) & 1u) ? ns : -1;
      if ((mask >> b) & 1u) bslot[ns++] = b;
    }
    for (; ns < 9; ++ns) bslot[ns] = -1;
  }
  __syncthreads();
  const int stride = nslot * D;
  for (int k2 = t; k2 < MF_NR * stride / 2; k2 += 256) {   // two complex values per 16-byte access
    const int k = 2 * k2, q = k / stride, kk = k - q * stride, sl2 = kk / D, j = kk - sl2 * D, r = r0 + q;
    const int b = bslot[sl2];
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    const long src = b >= 0 ? src9[b] : -1;
    if (src >= 0 && r < a.nrhs) {
      v = *reinterpret_cast<const float4*>(rho_in + r * VD + src * D + j);
      if (!first) {
        const cplx<float> al = alpha_s[q];
        const float4 qv = *reinterpret_cast<const float4*>(q_in + r * VD + src * D + j);
        v.x -= al.re * qv.x - al.im * qv.y;
        v.y -= al.re * qv.y + al.im * qv.x;
        v.z -= al.re * qv.z - al.im * qv.w;
        v.w -= al.re * qv.w + al.im * qv.z;
      }
    }
    *reinterpret_cast<float4*>(vst + k) = v;
  }
  __syncthreads();
  site_mv_mfma_pre<D>(Dc + y * 9L * D * D, vst, pre, stride, slot9);
  // wave q: right-hand sides r0 + q, r0 + q + 4, ...; lanes over rows
  const int wq = t >> 6, lane = t & 63;
  for (int q = wq; q < MF_NR; q += 4) {
    const int r = r0 + q;
    if (r >= a.nrhs) continue;   // uniform across the wave
    float qq = 0, qre = 0, qim = 0;
    if (lane < D) {
      const float mu = (float)mu_dev[r];
      const cplx<float> rho = vst[q * stride + lane];
      cplx<float> acc = site_mv_mfma_row<D>(vst, q, lane, stride);
      acc += (lane < D / 2 ? mu : -mu) * times_i(rho);
      const long o = r * VD + y * D + lane;
      q_out[o] = acc;
      rho_out[o] = rho;
      if (!first) cfma(z[o], alpha_s[q], rho_in[o]);
      qq = norm2(acc);
      const cplx<float> tq = cmulc(acc, rho);
      qre = tq.re;
      qim = tq.im;
    }
    qq = wave_sum(qq);
    qre = wave_sum(qre);
    qim = wave_sum(qim);
    if (lane == 0) {
      const long u = ((long)bi * cb.nbs + sl) * a.nrhs + r;
      part_out[3 * u] = qq;
      part_out[3 * u + 1] = qre;
      part_out[3 * u + 2] = qim;
    }
  }
}

// ------------------------------------------------------------------ level-1 SAP, one workgroup per block
// The whole colour's block solves in one launch: a workgroup of 8 waves
// takes one SAP block (at most 16 coarse sites) and 16 right-hand sides,
// forms the block residual rho = eta - D_c(mu) z on the matrix cores (the
// inputs of neighbouring blocks straight from memory), keeps rho of all
// the block's sites in LDS, and runs the MR steps with the step sizes from
// workgroup reductions (no per-step launches, no per-site partial sums in
// memory, the neighbours' rho read from LDS instead of being staged per
// site).  z is updated in place after every step.  Each wave owns up to
// two sites of the block; its D x 16 products stay in registers.
constexpr int SB_WAVES = 8;
constexpr int SB_SITES_PER_WAVE = 2;
constexpr int SB_MAX_SITES = SB_WAVES * SB_SITES_PER_WAVE;

// accr/acci += sum over the blocks b of mask of D_b(site) x input_b, with
// input_b(j0 + e) for this lane's right-hand side given by in(b, j0, v4);
// the D_c fragments of the next block load while the current one runs
template <int D, typename In>
TM_D void mf_site_accumulate(const unsigned* __restrict__ Du, unsigned mask, In in, mf_f4 (&accr)[D / 16],
                             mf_f4 (&acci)[D / 16]) {
  constexpr int MT = D / 16, KS = D / 16;
  const int l = threadIdx.x & 63, lk = l >> 4;
  unsigned an[KS][MT][4];
  int b = 0;
  while (b < 9 && !((mask >> b) & 1u)) ++b;
  if (b < 9) mf_load_block<D>(Du, b, an);
  while (b < 9) {
    unsigned ac[KS][MT][4];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e) ac[ks][mt][e] = an[ks][mt][e];
    int nb = b + 1;
    while (nb < 9 && !((mask >> nb) & 1u)) ++nb;
    if (nb < 9) mf_load_block<D>(Du, nb, an);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      cplx<float> v4[4];
      in(b, 16 * ks + 4 * lk, v4);
      const MfSplit bb = mf_split(v4);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        mf_s4 ar, ai;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ar[e] = (short)(ac[ks][mt][e] & 0xffffu);
          ai[e] = (short)(ac[ks][mt][e] >> 16);
        }
        mf_cmac(ar, ai, bb, accr[mt], acci[mt]);
      }
    }
    b = nb;
  }
}

template <int D>
__global__ void __launch_bounds__(SB_WAVES * 64, 1) k_sap1_block_mf(SapArgs a, const bf16pair* __restrict__ Dc,
                                                                      const cplx<float>* __restrict__ eta,
                                                                      cplx<float>* __restrict__ z,
                                                                      const double* __restrict__ mu_dev, int mr) {
  constexpr int MT = D / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<float>* rho = reinterpret_cast<cplx<float>*>(smem_raw);   // [site of the block][16][D]
  __shared__ double red[SB_WAVES][MF_NR][3];
  const CoarseGeom& g = a.g;
  const CBlk& cb = a.cb;
  const long VD = g.V * D;
  const int nbs = cb.nbs;
  const int ng = (a.nrhs + MF_NR - 1) / MF_NR;
  const int grp = blockIdx.x % ng, bi = blockIdx.x / ng;
  const int r0 = grp * MF_NR, blk = a.bl[bi];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  const int r = r0 + lr;
  const bool rv = r < a.nrhs;
  const float mu = rv ? (float)mu_dev[r] : 0.f;
  // this wave's sites of the block: sl = w + SB_WAVES * k
  long ys[SB_SITES_PER_WAVE];
  C4 lcs[SB_SITES_PER_WAVE];
#pragma unroll
  for (int k = 0; k < SB_SITES_PER_WAVE; ++k) {
    const int sl = w + SB_WAVES * k;
    ys[k] = -1;
    if (sl < nbs) {
      C4 c;
      cblk_site(cb, blk, sl, c, lcs[k]);
      ys[k] = cc_index(g, c);
    }
  }
  // ---- block residual: rho = eta - D_c(mu) z, all nine blocks
#pragma unroll
  for (int k = 0; k < SB_SITES_PER_WAVE; ++k) {
    if (ys[k] < 0) continue;   // uniform across the wave
    const long y = ys[k];
    const C4 c = cc_coords(g, y);
    long src[9];
    src[0] = y;
#pragma unroll
    for (int b = 1; b < 9; ++b) src[b] = cc_nbr(g, c, hop_mu(b), hop_step(b));
    mf_f4 accr[MT], acci[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) accr[mt] = acci[mt] = mf_f4{0.f, 0.f, 0.f, 0.f};
    const unsigned* Du = reinterpret_cast<const unsigned*>(Dc + y * 9L * D * D);
    mf_site_accumulate<D>(Du, 0x1FFu, [&](int b, int j0, cplx<float>* v4) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v4[e] = rv ? z[r * VD + src[b] * D + j0 + e] : mk(0.f, 0.f);
    }, accr, acci);
    const int sl = w + SB_WAVES * k;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * mt + 4 * lk + v;
        cplx<float> rh = mk(0.f, 0.f);
        if (rv) {
          cplx<float> acc = mk(accr[mt][v], acci[mt][v]);
          acc += (i < D / 2 ? mu : -mu) * times_i(z[r * VD + y * D + i]);
          rh = eta[r * VD + y * D + i] - acc;
        }
        rho[(sl * MF_NR + lr) * D + i] = rh;
      }
  }
  __syncthreads();
  // ---- MR steps on the block operator D_B
  for (int it = 0; it < mr; ++it) {
    mf_f4 qr_[SB_SITES_PER_WAVE][MT], qi_[SB_SITES_PER_WAVE][MT];
    float sqq = 0.f, sre = 0.f, sim = 0.f;
#pragma unroll
    for (int k = 0; k < SB_SITES_PER_WAVE; ++k) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) qr_[k][mt] = qi_[k][mt] = mf_f4{0.f, 0.f, 0.f, 0.f};
      if (ys[k] < 0) continue;
      const int sl = w + SB_WAVES * k;
      int nl[9];
      unsigned mask = 1u;
      nl[0] = sl;
#pragma unroll
      for (int b = 1; b < 9; ++b) {
        nl[b] = cblk_nbr(cb, lcs[k], hop_mu(b), hop_step(b));
        if (nl[b] >= 0) mask |= 1u << b;
      }
      const unsigned* Du = reinterpret_cast<const unsigned*>(Dc + ys[k] * 9L * D * D);
      mf_site_accumulate<D>(Du, mask, [&](int b, int j0, cplx<float>* v4) {
        const cplx<float>* p = rho + (nl[b] * MF_NR + lr) * D + j0;
#pragma unroll
        for (int e = 0; e < 4; ++e) v4[e] = p[e];
      }, qr_[k], qi_[k]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * mt + 4 * lk + v;
          const cplx<float> rh = rho[(sl * MF_NR + lr) * D + i];
          cplx<float> q = mk(qr_[k][mt][v], qi_[k][mt][v]);
          q += (i < D / 2 ? mu : -mu) * times_i(rh);
          qr_[k][mt][v] = q.re;
          qi_[k][mt][v] = q.im;
          acc_norm2(sqq, q);
          acc_dotc(sre, sim, q, rh);
        }
    }
    // the four lanes of a right-hand side (lk = 0..3), then the waves
    sqq += __shfl_xor(sqq, 16, 64);
    sre += __shfl_xor(sre, 16, 64);
    sim += __shfl_xor(sim, 16, 64);
    sqq += __shfl_xor(sqq, 32, 64);
    sre += __shfl_xor(sre, 32, 64);
    sim += __shfl_xor(sim, 32, 64);
    if (lk == 0) {
      red[w][lr][0] = sqq;
      red[w][lr][1] = sre;
      red[w][lr][2] = sim;
    }
    __syncthreads();   // every wave's products and reads of rho are done
    double dq = 0, dre = 0, dim = 0;
#pragma unroll
    for (int ww = 0; ww < SB_WAVES; ++ww) {
      dq += red[ww][lr][0];
      dre += red[ww][lr][1];
      dim += red[ww][lr][2];
    }
    const cplx<float> alpha = dq > 0 ? mk((float)(dre / dq), (float)(dim / dq)) : mk(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < SB_SITES_PER_WAVE; ++k) {
      if (ys[k] < 0) continue;
      const int sl = w + SB_WAVES * k;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * mt + 4 * lk + v;
          cplx<float>& rh = rho[(sl * MF_NR + lr) * D + i];
          if (rv) cfma(z[r * VD + ys[k] * D + i], alpha, rh);
          cfms(rh, alpha, mk(qr_[k][mt][v], qi_[k][mt][v]));
        }
    }
    __syncthreads();   // rho updated before the next step reads it; red free again
  }
}

// one launch per colour and sweep; false when the blocks do not fit (more
// than 16 sites or the LDS)
template <int D>
static bool sap_block_mf(const CoarseGeom& g, const CBlk& cb, const bf16pair* Dc, const cplx<float>* eta,
                         cplx<float>* z, int nrhs, const double* mu, const int* const bl[2], const int nb[2],
                         int sweeps, int mr, hipStream_t st) {
  // d = 64 needs more registers than a wave of this kernel has (it spills)
  const size_t lds = (size_t)cb.nbs * MF_NR * D * sizeof(cplx<float>);
  if (D > 48 || cb.nbs > SB_MAX_SITES || lds > 144 * 1024) return false;
  static bool attr = false;
  if (!attr) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sap1_block_mf<D>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, 144 * 1024));
    attr = true;
  }
  SapArgs a;
  a.g = g;
  a.cb = cb;
  a.nrhs = nrhs;
  const int ng = (nrhs + MF_NR - 1) / MF_NR;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int col = 0; col < 2; ++col) {
      if (nb[col] == 0) continue;
      a.bl = bl[col];
      hipLaunchKernelGGL((k_sap1_block_mf<D>), dim3((unsigned)(nb[col] * ng)), dim3(SB_WAVES * 64), lds, st, a, Dc,
                         eta, z, mu, mr);
    }
  return true;
}

template <int D, int MINB>
static void sap_fused_mf(const CoarseGeom& g, const CBlk& cb, const bf16pair* Dc, const cplx<float>* eta,
                         cplx<float>* z, int nrhs, const double* mu, const int* const bl[2], const int nb[2],
                         int sweeps, int mr, cplx<float>* const rho[2], cplx<float>* const q[2],
                         double* const part[2], hipStream_t st) {
  const size_t lds = (size_t)MF_NR * 9 * D * sizeof(cplx<float>);
  static bool attr = false;
  if (!attr && lds > 60 * 1024) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sap1_resid_mf<D, 1>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sap1_mr_mf<D, MINB>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  SapArgs a;
  a.g = g;
  a.cb = cb;
  a.nrhs = nrhs;
  // in-block neighbours a site can have: both along a direction whose block
  // extent is at least 3 (or that wraps), one along an extent of 2
  int nact = 1;
  for (int m = 0; m < 4; ++m) nact += (cb.NB[m] == 1 || cb.B[m] >= 3) ? 2 : (cb.B[m] == 2 ? 1 : 0);
  const int nslot = std::max(5, std::min(9, nact));
  const size_t lds_mr = (size_t)MF_NR * nslot * D * sizeof(cplx<float>);
  const int ng = (nrhs + MF_NR - 1) / MF_NR;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int col = 0; col < 2; ++col) {
      const int units = nb[col] * cb.nbs * ng;
      if (units == 0) continue;
      a.bl = bl[col];
      // the residual kernel's LDS allows two workgroups per CU anyway
      hipLaunchKernelGGL((k_sap1_resid_mf<D, 1>), dim3(units), dim3(256), lds, st, a, Dc, eta, z, rho[1], mu);
      for (int k = 0; k < mr; ++k) {
        const int in = (k + 1) & 1, out = k & 1;
        hipLaunchKernelGGL((k_sap1_mr_mf<D, MINB>), dim3(units), dim3(256), lds_mr, st, a, Dc, z, rho[in], q[in],
                           part[in], rho[out], q[out], part[out], mu, k == 0 ? 1 : 0, nslot);
      }
      if (mr > 0) {
        const int in = (mr - 1) & 1;
        hipLaunchKernelGGL((k_sap1_fin<float, D, MF_NR>), dim3(units), dim3(256), 0, st, a, z, rho[in], part[in]);
      }
    }
}

template <typename T, typename S, int D, int NR>
static void sap_fused(const CoarseGeom& g, const CBlk& cb, const SP<S>* Dc, const cplx<T>* eta, cplx<T>* z, int nrhs,
                      const double* mu, const int* const bl[2], const int nb[2], int sweeps, int mr,
                      cplx<T>* const rho[2], cplx<T>* const q[2], double* const part[2], hipStream_t st) {
  SapArgs a;
  a.g = g;
  a.cb = cb;
  a.nrhs = nrhs;
  const int ng = (nrhs + NR - 1) / NR;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int col = 0; col < 2; ++col) {
      const int units = nb[col] * cb.nbs * ng;
      if (units == 0) continue;
      a.bl = bl[col];
      // the residual goes to slot 1, the slot step 0 reads
      hipLaunchKernelGGL((k_sap1_resid<T, S, D, NR>), dim3(units), dim3(256), 0, st, a, Dc, eta, z, rho[1], mu);
      for (int k = 0; k < mr; ++k) {
        const int in = (k + 1) & 1, out = k & 1;
        hipLaunchKernelGGL((k_sap1_mr<T, S, D, NR>), dim3(units), dim3(256), 0, st, a, Dc, z, rho[in], q[in],
                           part[in], rho[out], q[out], part[out], mu, k == 0 ? 1 : 0);
      }
      if (mr > 0) {
        const int in = (mr - 1) & 1;
        hipLaunchKernelGGL((k_sap1_fin<T, D, NR>), dim3(units), dim3(256), 0, st, a, z, rho[in], part[in]);
      }
    }
}

template <typename T, typename S, int D>
static bool sap_mf(const CoarseGeom& g, const CBlk& cb, const SP<S>* Dc, const cplx<T>* eta, cplx<T>* z, int nrhs,
                   const double* mu, const int* const bl[2], const int nb[2], int sweeps, int mr,
                   cplx<T>* const rho[2], cplx<T>* const q[2], double* const part[2], hipStream_t st) {
  if constexpr (mf_ok<T, S, D>()) {
    const int tv = tune_get(TUNE_SAP1, D, g.V, nrhs);
    // variant 3: one workgroup per SAP block, the whole colour in one launch
    // (the rule's choice from 2 right-hand sides on where the blocks fit;
    // 32^3 x 64, one sweep: 12 RHS 0.54 ms against 1.32 ms for variant 2,
    // 2 RHS 0.50 ms against 0.86 ms on the vector ALU, 1 RHS 0.50 against 0.44)
    if ((tv >= 0 ? tv == 3 : nrhs >= 2) && sap_block_mf<D>(g, cb, Dc, eta, z, nrhs, mu, bl, nb, sweeps, mr, st)) {
      tune_used(TUNE_SAP1, 3);
      return true;
    }
    if (tv >= 0 ? tv >= 1 : nrhs >= 8) {
      // variant 2: register budget for four workgroups per CU (the rule
      // takes it from 4096 coarse sites on)
      const bool wide = tv >= 0 ? tv == 2 : g.V >= 4096;
      if (wide) sap_fused_mf<D, 4>(g, cb, Dc, eta, z, nrhs, mu, bl, nb, sweeps, mr, rho, q, part, st);
      else sap_fused_mf<D, 1>(g, cb, Dc, eta, z, nrhs, mu, bl, nb, sweeps, mr, rho, q, part, st);
      tune_used(TUNE_SAP1, wide ? 2 : 1);
      return true;
    }
  }
  tune_used(TUNE_SAP1, 0);
  return false;
}

template <typename T, typename S>
bool launch_sap_coarse_fused(const CoarseGeom& g, int d, const int blk[4], const SP<S>* Dc, const cplx<T>* eta,
                             cplx<T>* z, int nrhs, const double* mu_dev, const int* bl0, int n0, const int* bl1,
                             int n1, int sweeps, int mr_steps, cplx<T>* const rho[2], cplx<T>* const q[2],
                             double* const part[2], long part_cap, hipStream_t st) {
  if (!(d == 24 || d == 32 || d == 48 || d == 64)) return false;
  CBlk cb;
  cb.nbs = 1;
  for (int m = 0; m < 4; ++m) {
    cb.B[m] = blk[m];
    cb.NB[m] = g.L[m] / blk[m];
    cb.nbs *= blk[m];
  }
  const long units = (long)std::max(n0, n1) * cb.nbs * nrhs;
  if (units * 3 > part_cap || units > (1L << 30)) return false;
  const int* bl[2] = {bl0, bl1};
  const int nb[2] = {n0, n1};
  // one right-hand side per workgroup, or four (FP64: two) sharing each D_c load
  // eight or more right-hand sides with a bf16 D_c: 16 per workgroup on the matrix cores
#define SAP_CASE(DD)                                                                                   \
  if (nrhs == 1 && !(mf_ok<T, S, DD>() && tune_get(TUNE_SAP1, DD, g.V, 1) >= 1)) {                  \
    sap_fused<T, S, DD, 1>(g, cb, Dc, eta, z, nrhs, mu_dev, bl, nb, sweeps, mr_steps, rho, q, part, st);        \
    tune_used(TUNE_SAP1, 0);                                                                         \
  } else if (!sap_mf<T, S, DD>(g, cb, Dc, eta, z, nrhs, mu_dev, bl, nb, sweeps, mr_steps, rho, q, part, st))            \
    sap_fused<T, S, DD, sizeof(T) == 4 ? 4 : 2>(g, cb, Dc, eta, z, nrhs, mu_dev, bl, nb, sweeps, mr_steps, rho, q,     \
                                                  part, st);
  switch (d) {
    case 24: SAP_CASE(24) break;
    case 32: SAP_CASE(32) break;
    case 48: SAP_CASE(48) break;
    default: SAP_CASE(64) break;
  }
#undef SAP_CASE
  return true;
}

// ------------------------------------------------------------------ coarsest GMRES
// Barrier over the workgroups of a launch whose workgroups are all resident.  The counter only
// grows within a launch (epoch e waits for e * gridDim.x arrivals); the
// last workgroup to leave the kernel sets it back to zero for the next
// launch on the stream.  The wait is bounded: a timeout raises err and
// lets every wave run to the end.
TM_D void gbar(unsigned* ctr, unsigned& epoch, int* err) {
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(ctr, 1u);
    const unsigned target = epoch * gridDim.x;
    unsigned spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins == (1u << 26)) {
        atomicOr(err, 1);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}
TM_D void gbar_exit(unsigned* ctr) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(ctr + 1, 1u) == gridDim.x - 1) {
      atomicExch(ctr, 0u);
      atomicExch(ctr + 1, 0u);
    }
  }
}

struct CoopGmres {
  CoarseGeom g;
  int nrhs, m;
  double reltol;
};

struct CoopGmresWs {
  void* V;          // [(m+1)][nrhs][n] cplx<T>
  void* w;          // [nrhs][n]
  double* part1;    // [G][nrhs][m+2] complex: per-workgroup partial sums
  double* part2;    // [G][nrhs][m+2] complex
  double* R;        // [nrhs][m][m] complex: rotated Hessenberg, column j at [j][.]
  double* cs;       // [nrhs][m] complex (workgroup 0 only)
  double* sn;       // [nrhs][m]
  double* gv;       // [nrhs][m+1] complex
  double* tolabs;   // [nrhs]
  int* flags;       // [nrhs]
  int* kdone;       // [nrhs]
  unsigned* bar;    // [2] barrier counters (zero between launches)
  int* err;         // [1] barrier timeouts
  int* stat;        // [2] iterations summed over right-hand sides, launches
};

// Partial sums over the workgroup's own sites of conj(V_i) . w for the
// pairs (r, i), i < ni, plus (with with_norm) |w|^2 in slot ni; waves over
// pairs, lanes over the D rows, sites in a fixed order.
template <typename T, int D>
TM_D void own_dots(const cplx<T>* V, long vs, const cplx<T>* w, long n, int nrhs, int m, int ni, bool with_norm,
                   const int* flags, int nsites, double* part) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int per = ni + (with_norm ? 1 : 0);
  for (int q = wv; q < nrhs * per; q += 4) {
    const int r = q / per, i = q - r * per;
    double sre = 0, sim = 0;
    if (flags[r] && lane < D)
      for (int u = blockIdx.x; u < nsites; u += gridDim.x) {
        const long o = r * n + (long)u * D + lane;
        const cplx<T> cw = w[o];
        const cplx<T> av = i < ni ? V[(long)i * vs + o] : cw;
        sre += (double)av.re * cw.re + (double)av.im * cw.im;
        sim += (double)av.re * cw.im - (double)av.im * cw.re;
      }
    sre = wave_sum(sre);
    sim = wave_sum(sim);
    if (lane == 0) {
      double* p = part + 2L * (((long)blockIdx.x * nrhs + r) * (m + 2) + i);
      p[0] = sre;
      p[1] = sim;
    }
  }
}
// coef[r][i] = sum over workgroups of part[wg][r][i].  Four lanes share a
// pair, each summing every fourth workgroup, then combine by two
// shuffles: a fixed order, so every workgroup gets the same bits.
TM_D void all_reduce(const double* part, int nrhs, int m, int per, double* coef) {
  const int np = nrhs * per, sub = threadIdx.x & 3;
  for (int q0 = 0; q0 < np; q0 += 64) {
    const int q = q0 + (threadIdx.x >> 2);
    double sre = 0, sim = 0;
    if (q < np) {
      const int r = q / per, i = q - r * per;
      for (int wg = sub; wg < (int)gridDim.x; wg += 4) {
        const double* p = part + 2L * (((long)wg * nrhs + r) * (m + 2) + i);
        sre += p[0];
        sim += p[1];
      }
    }
    sre += __shfl_xor(sre, 1, 64);
    sim += __shfl_xor(sim, 1, 64);
    sre += __shfl_xor(sre, 2, 64);
    sim += __shfl_xor(sim, 2, 64);
    if (q < np && sub == 0) {
      const int r = q / per, i = q - r * per;
      coef[2 * (r * (m + 2) + i)] = sre;
      coef[2 * (r * (m + 2) + i) + 1] = sim;
    }
  }
  __syncthreads();
}
// w -= V c on the own sites (c from LDS, first ni columns)
template <typename T, int D>
TM_D void own_update(const cplx<T>* V, long vs, cplx<T>* w, long n, int nrhs, int m, int ni, const double* coef,
                     const int* flags, int nsites) {
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    for (int k = threadIdx.x; k < nrhs * D; k += blockDim.x) {
      const int r = k / D, i = k - r * D;
      if (!flags[r]) continue;
      const long o = r * n + (long)u * D + i;
      cplx<T> acc = w[o];
      for (int l = 0; l < ni; ++l)
        cfma(acc, mk<T>((T)(-coef[2 * (r * (m + 2) + l)]), (T)(-coef[2 * (r * (m + 2) + l) + 1])),
             V[(long)l * vs + o]);
      w[o] = acc;
    }
}
// |h_{j+1,j}| from the second pass: |w|^2 - |c2|^2
TM_D double new_norm(const double* c2r, int j) {
  double h2 = c2r[2 * (j + 1)];
  for (int l = 0; l <= j; ++l) h2 -= c2r[2 * l] * c2r[2 * l] + c2r[2 * l + 1] * c2r[2 * l + 1];
  return h2 > 0 ? sqrt(h2) : 0.0;
}

// GMRES(m) from x = 0 for D_c(mu_r) x_r = b_r, stopping a right-hand side
// when its implicit residual <= reltol * ||b_r||.  Classical Gram-Schmidt
// with one re-orthogonalisation pass; the norm of the new direction comes
// from |w|^2 - |c2|^2 after the second pass.  Workgroup 0 applies the
// Givens rotations; every workgroup solves the small triangular system at
// the end for its own sites.
template <typename T, typename S, int D>
__global__ void __launch_bounds__(256) k_coarsest_gmres(CoopGmres a, const SP<S>* __restrict__ Dc,
                                                        const cplx<T>* __restrict__ b, cplx<T>* x,
                                                        const double* __restrict__ mu_dev, CoopGmresWs ws) {
  __shared__ cplx<T> vst[9 * D];
  __shared__ cplx<T> red[SiteMV<D>::KS * D];
  __shared__ int any_active;
  extern __shared__ double coef[];   // c1 [nrhs][m+2], c2 [nrhs][m+2] complex; y reuses c1
  const CoarseGeom& g = a.g;
  const int nrhs = a.nrhs, m = a.m;
  const long n = g.V * D;
  const int nsites = (int)g.V;
  cplx<T>* V = static_cast<cplx<T>*>(ws.V);
  cplx<T>* w = static_cast<cplx<T>*>(ws.w);
  const long vs = (long)nrhs * n;
  double* c1 = coef;
  double* c2 = coef + 2 * nrhs * (m + 2);
  const int t = threadIdx.x;
  unsigned epoch = 0;

  // ||b_r||^2 partials in part1 slot 0
  {
    const int lane = t & 63, wv = t >> 6;
    for (int r = wv; r < nrhs; r += 4) {
      double s2 = 0;
      if (lane < D)
        for (int u = blockIdx.x; u < nsites; u += gridDim.x) s2 += (double)norm2(b[r * n + (long)u * D + lane]);
      s2 = wave_sum(s2);
      if (lane == 0) {
        double* p = ws.part1 + 2L * (((long)blockIdx.x * nrhs + r) * (m + 2));
        p[0] = s2;
        p[1] = 0;
      }
    }
  }
  gbar(ws.bar, epoch, ws.err);
  all_reduce(ws.part1, nrhs, m, 1, c1);
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    for (int k = t; k < nrhs * D; k += 256) {
      const int r = k / D, i = k - r * D;
      const double bt = sqrt(c1[2 * r * (m + 2)]);
      const long o = r * n + (long)u * D + i;
      V[o] = bt > 0 ? (T)(1.0 / bt) * b[o] : mk<T>(0, 0);
    }
  if (blockIdx.x == 0)
    for (int r = t; r < nrhs; r += 256) {
      const double bt = sqrt(c1[2 * r * (m + 2)]);
      ws.gv[2 * r * (m + 1)] = bt;
      ws.gv[2 * r * (m + 1) + 1] = 0;
      ws.tolabs[r] = a.reltol * bt;
      ws.kdone[r] = 0;
      ws.flags[r] = (bt > 0 && bt < 1e300) ? 1 : 0;
    }
  gbar(ws.bar, epoch, ws.err);

  for (int j = 0; j < m; ++j) {
    if (t == 0) {
      int any = 0;
      for (int r = 0; r < nrhs; ++r) any |= ws.flags[r];
      any_active = any;
    }
    __syncthreads();
    if (!any_active) break;   // same in every workgroup: flags change only before a barrier
    const cplx<T>* vj = V + (long)j * vs;
    // w = D_c(mu) v_j on the own sites
    for (int u = blockIdx.x; u < nsites; u += gridDim.x) {
      const C4 c = cc_coords(g, u);
      for (int r = 0; r < nrhs; ++r) {
        if (!ws.flags[r]) continue;   // uniform across the workgroup
        const cplx<T>* vr = vj + r * n;
        for (int k = t; k < 9 * D; k += 256) {
          const int bb = k / D, jj = k - bb * D;
          const long src = bb == 0 ? u : cc_nbr(g, c, hop_mu(bb), hop_step(bb));
          vst[k] = vr[src * D + jj];
        }
        __syncthreads();
        site_mv<T, S, D>(Dc + (long)u * 9L * D * D, vst, 0x1FFu, red);
        if (t < D) {
          const T mu = (T)mu_dev[r];
          cplx<T> acc = site_mv_row<T, D>(red, t);
          acc += (t < D / 2 ? mu : -mu) * times_i(vst[t]);
          w[r * n + (long)u * D + t] = acc;
        }
        __syncthreads();
      }
    }
    // first Gram-Schmidt pass
    own_dots<T, D>(V, vs, w, n, nrhs, m, j + 1, false, ws.flags, nsites, ws.part1);
    gbar(ws.bar, epoch, ws.err);
    all_reduce(ws.part1, nrhs, m, j + 1, c1);
    own_update<T, D>(V, vs, w, n, nrhs, m, j + 1, c1, ws.flags, nsites);
    __syncthreads();
    // second pass, with |w|^2 in slot j + 1
    own_dots<T, D>(V, vs, w, n, nrhs, m, j + 1, true, ws.flags, nsites, ws.part2);
    gbar(ws.bar, epoch, ws.err);
    all_reduce(ws.part2, nrhs, m, j + 2, c2);
    own_update<T, D>(V, vs, w, n, nrhs, m, j + 1, c2, ws.flags, nsites);
    __syncthreads();
    cplx<T>* vn = V + (long)(j + 1) * vs;
    for (int u = blockIdx.x; u < nsites; u += gridDim.x)
      for (int k = t; k < nrhs * D; k += 256) {
        const int r = k / D, i = k - r * D;
        if (!ws.flags[r]) continue;
        const double hn = new_norm(c2 + 2 * r * (m + 2), j);
        const long o = r * n + (long)u * D + i;
        vn[o] = hn > 0 ? (T)(1.0 / hn) * w[o] : mk<T>(0, 0);
      }
    if (blockIdx.x == 0)
      for (int r = t; r < nrhs; r += 256) {
        if (!ws.flags[r]) continue;
        double* Rc = ws.R + 2L * ((long)r * m * m + (long)j * m);   // column j
        double* cs = ws.cs + 2L * r * m;
        double* sn = ws.sn + (long)r * m;
        double* gg = ws.gv + 2L * r * (m + 1);
        const double* h1 = c1 + 2 * r * (m + 2);
        const double* h2 = c2 + 2 * r * (m + 2);
        const double hn = new_norm(h2, j);
        // previous rotations [[c, s], [-s, conj(c)]] (s real) on column j
        double ar = h1[0] + h2[0], ai = h1[1] + h2[1];
        for (int i = 0; i < j; ++i) {
          const double br = h1[2 * (i + 1)] + h2[2 * (i + 1)], bi = h1[2 * (i + 1) + 1] + h2[2 * (i + 1) + 1];
          const double cr = cs[2 * i], ci = cs[2 * i + 1], s = sn[i];
          Rc[2 * i] = cr * ar - ci * ai + s * br;
          Rc[2 * i + 1] = cr * ai + ci * ar + s * bi;
          const double ur = -s * ar + (cr * br + ci * bi);
          const double ui = -s * ai + (cr * bi - ci * br);
          ar = ur;
          ai = ui;
        }
        const double den = sqrt(ar * ar + ai * ai + hn * hn);
        if (!(den > 0) || den != den) {
          ws.flags[r] = 0;
          continue;
        }
        const double cr = ar / den, ci = -ai / den, s = hn / den;
        cs[2 * j] = cr;
        cs[2 * j + 1] = ci;
        sn[j] = s;
        Rc[2 * j] = den;
        Rc[2 * j + 1] = 0;
        const double gr = gg[2 * j], gi = gg[2 * j + 1];
        gg[2 * (j + 1)] = -s * gr;
        gg[2 * (j + 1) + 1] = -s * gi;
        gg[2 * j] = cr * gr - ci * gi;
        gg[2 * j + 1] = cr * gi + ci * gr;
        ws.kdone[r] = j + 1;
        const double res = s * sqrt(gr * gr + gi * gi);
        if (res <= ws.tolabs[r] || hn <= 1e-15 * den || j + 1 >= m) ws.flags[r] = 0;
      }
    gbar(ws.bar, epoch, ws.err);
  }
  // y = R^-1 g (every workgroup, into c1), then x = V y on the own sites
  for (int r = t; r < nrhs; r += 256) {
    const int k = ws.kdone[r];
    const double* Rr = ws.R + 2L * r * m * m;
    const double* gg = ws.gv + 2L * r * (m + 1);
    double* yv = c1 + 2 * r * (m + 2);
    for (int i = k - 1; i >= 0; --i) {
      double sr = gg[2 * i], si = gg[2 * i + 1];
      for (int l = i + 1; l < k; ++l) {
        const double hr = Rr[2 * (l * m + i)], hi = Rr[2 * (l * m + i) + 1];
        sr -= hr * yv[2 * l] - hi * yv[2 * l + 1];
        si -= hr * yv[2 * l + 1] + hi * yv[2 * l];
      }
      const double dr = Rr[2 * (i * m + i)], di = Rr[2 * (i * m + i) + 1];
      const double dd = dr * dr + di * di;
      yv[2 * i] = (sr * dr + si * di) / dd;
      yv[2 * i + 1] = (si * dr - sr * di) / dd;
    }
  }
  if (blockIdx.x == 0 && t == 0) {
    int its = 0;
    for (int r = 0; r < nrhs; ++r) its += ws.kdone[r];
    atomicAdd(ws.stat, its);
    atomicAdd(ws.stat + 1, 1);
  }
  __syncthreads();
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    for (int k = t; k < nrhs * D; k += 256) {
      const int r = k / D, i = k - r * D;
      const int kd = ws.kdone[r];
      const double* yv = c1 + 2 * r * (m + 2);
      const long o = r * n + (long)u * D + i;
      cplx<T> acc = mk<T>(0, 0);
      for (int l = 0; l < kd; ++l) cfma(acc, mk<T>((T)yv[2 * l], (T)yv[2 * l + 1]), V[(long)l * vs + o]);
      x[o] = acc;
    }
  gbar_exit(ws.bar);
}

// ------------------------------------------------------------------ coarsest GMRES, one site per workgroup
// Single right-hand side, FP32 arithmetic on a 16-bit D_c, at most 256
// coarse sites.  Workgroup u owns site u and keeps:
//  * the nine D_c blocks of the site in LDS for the whole solve;
//  * the site's rows of the Krylov basis v_i and of p_i = (v_i - sum_{l<i}
//    R_li p_l) / R_ii in registers, wave w holding i = w (mod 4);
//  * its rows of x = sum_i g_i p_i, updated as soon as column i of the
//    rotated Hessenberg R and the rotated g_i are final, so no triangular
//    solve is left at the end;
//  * its own copy of the Givens rotations: every workgroup rotates the
//    same Hessenberg column from the same sums, so convergence decisions
//    and R need no broadcast.
// Only the newest basis vector and per-workgroup partial sums (float
// pairs, [pair][workgroup]) cross workgroups; both are written with
// agent-scope stores so that the barrier's cache write-back finds little.
struct SiteGmres {
  CoarseGeom g;
  int m;
  double reltol;
};
struct SiteGmresWs {
  cplx<float>* vg0;   // [n] newest basis vector, even j
  cplx<float>* vg1;   // [n] odd j
  float* part1;       // [m+2][Gp] complex float, Gp = G rounded up to even
  float* part2;       // [m+2][Gp]
  unsigned* bar;      // [2]
  int* err;           // [1]
  int* stat;          // [2] iterations, launches
  int* reorth;        // [1] second Gram-Schmidt passes
};

constexpr int SITE_SLOTS = 32;   // basis vectors per wave: m + 1 <= 128

TM_D void st_agent(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// sums[q] (q < P) = sum over workgroups of part[q][wg] (complex float).
// L lanes share a pair (the largest power of two with L * P <= 256); a lane
// loads two workgroups' values per 16-byte access, eight accesses in
// flight; shuffles combine the lanes.  Identical bits in every workgroup.
TM_D void gather_sums(const float* __restrict__ part, int P, int Gp, double* out) {
  int L = 64;
  while (L > 1 && L * P > 256) L >>= 1;
  const int t = threadIdx.x, sub = t & (L - 1), slot = t / L, nslot = 256 / L;
  const int G2 = Gp >> 1;   // float4 = two workgroups
  for (int q0 = 0; q0 < P; q0 += nslot) {
    const int q = q0 + slot;
    double re[8], im[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) re[k] = im[k] = 0;
    if (q < P) {
      const float4* pp = reinterpret_cast<const float4*>(part) + (long)q * G2;
      int w2 = sub;
      for (; w2 + 7 * L < G2; w2 += 8 * L) {
        float4 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = pp[w2 + k * L];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          re[k] += (double)v[k].x + (double)v[k].z;
          im[k] += (double)v[k].y + (double)v[k].w;
        }
      }
      for (; w2 < G2; w2 += L) {
        const float4 v = pp[w2];
        re[0] += (double)v.x + (double)v.z;
        im[0] += (double)v.y + (double)v.w;
      }
    }
    double sr = ((re[0] + re[1]) + (re[2] + re[3])) + ((re[4] + re[5]) + (re[6] + re[7]));
    double si = ((im[0] + im[1]) + (im[2] + im[3])) + ((im[4] + im[5]) + (im[6] + im[7]));
    for (int o = 1; o < L; o <<= 1) {
      sr += __shfl_xor(sr, o, 64);
      si += __shfl_xor(si, o, 64);
    }
    if (q < P && sub == 0) {
      out[2 * q] = sr;
      out[2 * q + 1] = si;
    }
  }
  __syncthreads();
}

template <typename S, int D>
__global__ void __launch_bounds__(256) k_coarsest_gmres_site(SiteGmres a, const SP<S>* __restrict__ Dc,
                                                             const cplx<float>* __restrict__ b,
                                                             cplx<float>* __restrict__ x,
                                                             const double* __restrict__ mu_dev, SiteGmresWs ws) {
  using cf = cplx<float>;
  constexpr int KQ = 9 * D / 4;   // terms per wave in the matrix-vector product
  __shared__ cf vst[9 * D];
  __shared__ cf comb[4][64];
  __shared__ cf wl[64];
  __shared__ cf pl[64];
  __shared__ double c1[2 * (4 * SITE_SLOTS + 1)];
  __shared__ double c2[2 * (4 * SITE_SLOTS + 1)];
  __shared__ double rcol[2 * 4 * SITE_SLOTS];   // rotated column of the last iteration
  __shared__ double s_g[2];                     // its final rotated g
  __shared__ int s_flag, s_kd;
  extern __shared__ __align__(16) unsigned char dyn[];
  SP<S>* dcl = reinterpret_cast<SP<S>*>(dyn);
  const CoarseGeom& g = a.g;
  const int m = a.m, G = gridDim.x, Gp = (G + 1) & ~1, u = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const float mu = (float)mu_dev[0];
  unsigned epoch = 0;
  int n_reorth = 0;
  cf Vr[SITE_SLOTS], Pr[SITE_SLOTS];
#pragma unroll
  for (int s = 0; s < SITE_SLOTS; ++s) Vr[s] = Pr[s] = mk<float>(0, 0);
  // wave 0: x rows, the newest basis vector, and v_i of the column i whose
  // p_i is formed at the top of the next iteration
  cf xacc = mk<float>(0, 0), vcur = mk<float>(0, 0), vfin = mk<float>(0, 0);
  // Givens state (wave 0): rotation i in lane i % 64, slot i / 64
  double csr0 = 0, csi0 = 0, sn0 = 0, csr1 = 0, csi1 = 0, sn1 = 0, gre = 0, gim = 0, tolabs = 0;

  {
    const Quad<S>* src = reinterpret_cast<const Quad<S>*>(Dc + (long)u * 9L * D * D);
    Quad<S>* dst = reinterpret_cast<Quad<S>*>(dcl);
    for (int k = t; k < 9 * D * D / 4; k += 256) dst[k] = src[k];
  }
  if (u == 0 && (G & 1) && t < 2 * (m + 2)) {
    // with an odd workgroup count every pair's padding slot reads as zero
    const int q = t >> 1;
    float* p = (t & 1) ? ws.part2 : ws.part1;
    st_agent(p + 2L * ((long)q * Gp + G), 0.f);
    st_agent(p + 2L * ((long)q * Gp + G) + 1, 0.f);
  }
  if (t < 64) {
    const cf bv = lane < D ? b[(long)u * D + lane] : mk<float>(0, 0);
    vcur = bv;
    float s2 = norm2(bv);
    s2 = wave_sum(s2);
    if (lane == 0) {
      st_agent(ws.part1 + 2L * u, s2);
      st_agent(ws.part1 + 2L * u + 1, 0.f);
    }
  }
  gbar(ws.bar, epoch, ws.err);
  gather_sums(ws.part1, 1, Gp, c1);
  {
    const double beta = sqrt(c1[0]);
    const bool ok = beta > 0 && beta < 1e300;
    if (t < 64) {
      vcur = ok ? (float)(1.0 / beta) * vcur : mk<float>(0, 0);
      Vr[0] = vcur;
      if (lane < D) {
        float* vp = reinterpret_cast<float*>(ws.vg0 + (long)u * D + lane);
        st_agent(vp, vcur.re);
        st_agent(vp + 1, vcur.im);
      }
      gre = beta;
      tolabs = a.reltol * beta;
    }
    if (t == 0) {
      s_flag = ok ? 1 : 0;
      s_kd = 0;
    }
  }
  gbar(ws.bar, epoch, ws.err);

  for (int j = 0;; ++j) {
    const int kd = s_kd;   // set by this workgroup's own rotation before the barrier
    // column j-1 final: p_{j-1} = (v_{j-1} - sum_{l<j-1} R_{l,j-1} p_l) / R_{j-1,j-1}, x += g_{j-1} p_{j-1}
    if (j > 0 && kd >= j) {
      const int i = j - 1;
      cf acc = mk<float>(0, 0);
#pragma unroll
      for (int s = 0; s < SITE_SLOTS; ++s) {
        const int l = 4 * s + wv;
        if (4 * s >= i) break;
        if (l < i) cfma(acc, mk<float>((float)rcol[2 * l], (float)rcol[2 * l + 1]), Pr[s]);
      }
      comb[wv][lane] = acc;
      __syncthreads();
      if (t < 64) {
        const cf sum = (comb[0][lane] + comb[1][lane]) + (comb[2][lane] + comb[3][lane]);
        const double dr = rcol[2 * i], di = rcol[2 * i + 1], dd = dr * dr + di * di;
        const cf num = vfin - sum;
        // num / R_ii
        const cf pv = mk<float>((float)((num.re * dr + num.im * di) / dd), (float)((num.im * dr - num.re * di) / dd));
        pl[lane] = pv;
        cfma(xacc, mk<float>((float)s_g[0], (float)s_g[1]), pv);
      }
      __syncthreads();
      if (wv == (i & 3)) {
#pragma unroll
        for (int s = 0; s < SITE_SLOTS; ++s)
          if (s == (i >> 2)) Pr[s] = pl[lane];
      }
    }
    if (j == m || !s_flag) break;   // same in every workgroup

    // w = D_c(mu) v_j on the own site: stage the nine input vectors, then
    // rows over lanes and a quarter of the 9*D terms per wave
    const cf* vj = (j & 1) ? ws.vg1 : ws.vg0;
    {
      const C4 c = cc_coords(g, u);
      for (int k = t; k < 9 * D; k += 256) {
        const int bb = k / D, jj = k - bb * D;
        const long src = bb == 0 ? u : cc_nbr(g, c, hop_mu(bb), hop_step(bb));
        vst[k] = vj[src * D + jj];
      }
    }
    __syncthreads();
    if (lane < D) {
      cf acc = mk<float>(0, 0);
      const int k0 = wv * KQ;
#pragma unroll 8
      for (int k = k0; k < k0 + KQ; ++k) cfma(acc, Store<S>::template cvt<float>(dcl[k * D + lane]), vst[k]);
      comb[wv][lane] = acc;
    }
    __syncthreads();
    if (t < D) {
      cf w = (comb[0][t] + comb[1][t]) + (comb[2][t] + comb[3][t]);
      w += (t < D / 2 ? mu : -mu) * times_i(vst[t]);
      wl[t] = w;
    }
    __syncthreads();

    // Classical Gram-Schmidt with |w|^2 in the same reduction; a second pass
    // only where the first cancelled more than one digit of w
    // (||w - V c|| < ||w|| / 10, a DGKS-type test with a threshold of 0.1: the
    // short coarsest solves, at most a few dozen steps to a relative 1e-1,
    // do not need the classical 1/sqrt 2).  Every workgroup takes the same
    // decision from the same sums.
    double hn = 0;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      float* part = pass ? ws.part2 : ws.part1;
      double* cc = pass ? c2 : c1;
      const cf wv_l = lane < D ? wl[lane] : mk<float>(0, 0);
#pragma unroll
      for (int s = 0; s < SITE_SLOTS; ++s) {
        const int i = 4 * s + wv;
        if (4 * s > j) break;
        if (i <= j) {
          const cf d = cmulc(Vr[s], wv_l);
          const float dre = wave_sum(d.re), dim = wave_sum(d.im);
          if (lane == 0) {
            st_agent(part + 2L * ((long)i * Gp + u), dre);
            st_agent(part + 2L * ((long)i * Gp + u) + 1, dim);
          }
        }
      }
      if (wv == 0) {
        const float n2 = wave_sum(norm2(wv_l));
        if (lane == 0) {
          st_agent(part + 2L * ((long)(j + 1) * Gp + u), n2);
          st_agent(part + 2L * ((long)(j + 1) * Gp + u) + 1, 0.f);
        }
      }
      gbar(ws.bar, epoch, ws.err);
      gather_sums(part, j + 2, Gp, cc);
      cf acc = mk<float>(0, 0);
#pragma unroll
      for (int s = 0; s < SITE_SLOTS; ++s) {
        const int i = 4 * s + wv;
        if (4 * s > j) break;
        if (i <= j) cfma(acc, mk<float>((float)cc[2 * i], (float)cc[2 * i + 1]), Vr[s]);
      }
      comb[wv][lane] = acc;
      __syncthreads();
      if (t < D) wl[t] = wl[t] - ((comb[0][t] + comb[1][t]) + (comb[2][t] + comb[3][t]));
      // |w - V c|^2 = |w|^2 - |c|^2 (V orthonormal)
      const double w2 = cc[2 * (j + 1)];
      double r2 = w2;
      for (int l = 0; l <= j; ++l) r2 -= cc[2 * l] * cc[2 * l] + cc[2 * l + 1] * cc[2 * l + 1];
      hn = r2 > 0 ? sqrt(r2) : 0.0;
      if (pass == 0 && r2 >= 0.01 * w2) {
        for (int e = t; e < 2 * (j + 2); e += 256) c2[e] = 0;
        __syncthreads();
        break;   // same decision in every workgroup
      }
      if (pass == 0) n_reorth++;
      __syncthreads();
    }
    {
      const cf vn = (lane < D && hn > 0) ? (float)(1.0 / hn) * wl[lane] : mk<float>(0, 0);
      if (wv == ((j + 1) & 3)) {
#pragma unroll
        for (int s = 0; s < SITE_SLOTS; ++s)
          if (s == ((j + 1) >> 2)) Vr[s] = vn;
      }
      if (t < 64) {
        vfin = vcur;
        vcur = vn;
        if (lane < D) {
          float* vp = reinterpret_cast<float*>(((j & 1) ? ws.vg0 : ws.vg1) + (long)u * D + lane);
          st_agent(vp, vn.re);
          st_agent(vp + 1, vn.im);
        }
      }
    }
    // Givens rotations (wave 0 of every workgroup, identical inputs)
    if (t < 64) {
      double ar = c1[0] + c2[0], ai = c1[1] + c2[1];
      for (int i = 0; i < j; ++i) {
        const bool hi = i >= 64;
        const double cr = __shfl(hi ? csr1 : csr0, i & 63, 64);
        const double ci = __shfl(hi ? csi1 : csi0, i & 63, 64);
        const double sn = __shfl(hi ? sn1 : sn0, i & 63, 64);
        const double br = c1[2 * (i + 1)] + c2[2 * (i + 1)], bi = c1[2 * (i + 1) + 1] + c2[2 * (i + 1) + 1];
        if (t == 0) {
          rcol[2 * i] = cr * ar - ci * ai + sn * br;
          rcol[2 * i + 1] = cr * ai + ci * ar + sn * bi;
        }
        const double ur = -sn * ar + (cr * br + ci * bi);
        const double ui = -sn * ai + (cr * bi - ci * br);
        ar = ur;
        ai = ui;
      }
      const double den = sqrt(ar * ar + ai * ai + hn * hn);
      if (!(den > 0) || den != den) {
        if (t == 0) s_flag = 0;
      } else {
        const double cr = ar / den, ci = -ai / den, sn = hn / den;
        if (lane == (j & 63)) {
          if (j >= 64) { csr1 = cr; csi1 = ci; sn1 = sn; }
          else { csr0 = cr; csi0 = ci; sn0 = sn; }
        }
        const double res = sn * sqrt(gre * gre + gim * gim);
        if (t == 0) {
          rcol[2 * j] = den;
          rcol[2 * j + 1] = 0;
          s_g[0] = cr * gre - ci * gim;
          s_g[1] = cr * gim + ci * gre;
          s_kd = j + 1;
          if (res <= tolabs || hn <= 1e-15 * den || j + 1 >= m) s_flag = 0;
        }
        const double ngr = -sn * gre, ngi = -sn * gim;
        gre = ngr;
        gim = ngi;
      }
    }
    gbar(ws.bar, epoch, ws.err);
  }
  if (t < D) x[(long)u * D + t] = xacc;
  if (u == 0 && t == 0) {
    atomicAdd(ws.stat, s_kd);
    atomicAdd(ws.stat + 1, 1);
    atomicAdd(ws.reorth, n_reorth);
  }
  gbar_exit(ws.bar);
}

// Workgroups of the shared-site coarsest GMRES (several sites per
// workgroup); TMAMG_COARSEST_WG overrides the default.
static int coarsest_shared_groups() {
  static int cap = -1;
  if (cap < 0) {
    const char* e = getenv("TMAMG_COARSEST_WG");
    cap = e ? std::max(1, std::min(256, atoi(e))) : 64;
  }
  return cap;
}

// upper bound of the workgroup count, which sizes the partial-sum arrays
int coarsest_groups(long nsites) { return (int)std::max<long>(1, std::min<long>(256, nsites)); }

size_t coarsest_ws_doubles(int nrhs, int m, int G) {
  return 2 * 2 * (size_t)G * nrhs * (m + 2) + (size_t)nrhs * (2 * (size_t)m * m + 2 * m + m + 2 * (m + 1) + 1);
}
// ints: barrier counters [0, 1], timeout flag [2], statistics [3, 4],
// flags and iteration counts of the right-hand sides from [8]
size_t coarsest_ws_ints(int nrhs) { return 2 * (size_t)nrhs + 8; }

// The persistent kernels synchronise through their own barrier, so every
// workgroup must be resident at once.  They are launched as ordinary
// kernels (no separate cooperative queue) after checking that the grid
// fits the device at the kernel's occupancy; the barrier's bounded wait
// still lets every wave finish if that ever fails to hold.
static bool grid_fits(const void* kern, int G, size_t dyn) {
  int dev = 0, per_cu = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, dyn) != hipSuccess) return false;
  return (long)per_cu * ncu >= G;
}

static hipError_t launch_resident(const void* kern, int G, void** args, size_t dyn, hipStream_t st) {
  if (!grid_fits(kern, G, dyn)) return hipErrorCooperativeLaunchTooLarge;
  return hipLaunchKernel(kern, dim3(G), dim3(256), args, dyn, st);
}

template <typename T, typename S, int D>
static hipError_t gmres_launch(CoopGmres a, size_t coef_bytes, const SP<S>* Dc, const cplx<T>* b, cplx<T>* x,
                               const double* mu_dev, CoopGmresWs ws, hipStream_t st) {
  const int G = (int)std::min<long>(a.g.V, coarsest_shared_groups());
  const void* kern = reinterpret_cast<const void*>(&k_coarsest_gmres<T, S, D>);
  if (coef_bytes > 65536) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)coef_bytes);
    if (e != hipSuccess) return e;
  }
  void* args[] = {&a, (void*)&Dc, (void*)&b, (void*)&x, (void*)&mu_dev, &ws};
  return launch_resident(kern, G, args, coef_bytes, st);
}

template <typename S, int D>
static hipError_t site_gmres_launch(const SiteGmres& a, const SP<S>* Dc, const cplx<float>* b, cplx<float>* x,
                                    const double* mu_dev, const SiteGmresWs& ws, hipStream_t st) {
  const void* kern = reinterpret_cast<const void*>(&k_coarsest_gmres_site<S, D>);
  const size_t dyn = 9 * (size_t)D * D * sizeof(SP<S>);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
    attr = true;
  }
  SiteGmres aa = a;
  SiteGmresWs ww = ws;
  void* args[] = {&aa, (void*)&Dc, (void*)&b, (void*)&x, (void*)&mu_dev, &ww};
  return launch_resident(kern, (int)a.g.V, args, dyn, st);
}

// FP32 over a 16-bit D_c, at most 256 sites, one launch per right-hand side
// (up to two: one launch at 300 us per RHS on the 24^3x48 hierarchy beats
// the shared-site kernel's 750 us for a pair)
template <typename T, typename S>
static bool try_site_gmres(const CoarseGeom& g, int d, const SP<S>* Dc, const cplx<T>* b, cplx<T>* x, int nrhs,
                           const double* mu_dev, int m, double reltol, cplx<T>* Vbasis, double* dws, size_t dws_cap,
                           int* iws, size_t iws_cap, hipStream_t st) {
  if constexpr (!std::is_same<T, float>::value || sizeof(SP<S>) != 4) {
    return false;
  } else {
    if (nrhs < 1 || nrhs > 2 || g.V > 256 || m + 1 > 4 * SITE_SLOTS) return false;
    const int G = (int)g.V;
    const int Gp = (G + 1) & ~1;
    if ((size_t)2 * Gp * (m + 2) > dws_cap || iws_cap < 8) return false;
    SiteGmres a;
    a.g = g;
    a.m = m;
    a.reltol = reltol;
    SiteGmresWs ws;
    ws.vg0 = Vbasis;
    ws.vg1 = Vbasis + g.V * d;
    float* fp = reinterpret_cast<float*>(dws);
    ws.part1 = fp;
    ws.part2 = fp + 2 * (size_t)Gp * (m + 2);
    ws.bar = reinterpret_cast<unsigned*>(iws);
    ws.err = iws + 2;
    ws.stat = iws + 3;
    ws.reorth = iws + 7;
    // the launches share the workspace in stream order; a failure leaves x to
    // the caller's fallback, which solves every right-hand side again
    const long n = g.V * (long)d;
    for (int r = 0; r < nrhs; ++r) {
      const cplx<float>* br = b + r * n;
      cplx<float>* xr = x + r * n;
      hipError_t e;
      switch (d) {
        case 24: e = site_gmres_launch<S, 24>(a, Dc, br, xr, mu_dev + r, ws, st); break;
        case 32: e = site_gmres_launch<S, 32>(a, Dc, br, xr, mu_dev + r, ws, st); break;
        case 48: e = site_gmres_launch<S, 48>(a, Dc, br, xr, mu_dev + r, ws, st); break;
        case 64: e = site_gmres_launch<S, 64>(a, Dc, br, xr, mu_dev + r, ws, st); break;
        default: return false;
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
    }
    return true;
  }
}

template <typename T, typename S>
bool launch_coarsest_gmres(const CoarseGeom& g, int d, const SP<S>* Dc, const cplx<T>* b, cplx<T>* x, int nrhs,
                           const double* mu_dev, int m, double reltol, cplx<T>* Vbasis, cplx<T>* w, double* dws,
                           size_t dws_cap, int* iws, size_t iws_cap, hipStream_t st) {
  if (!(d == 24 || d == 32 || d == 48 || d == 64) || m < 1) return false;
  if (try_site_gmres<T, S>(g, d, Dc, b, x, nrhs, mu_dev, m, reltol, Vbasis, dws, dws_cap, iws, iws_cap, st))
    return true;
  // the shared-site kernel serialises right-hand sides inside a workgroup:
  // wide batches go to the generic Krylov path; so do large coarsest
  // lattices, whose D_c no longer stays in cache between iterations and
  // which its few resident workgroups would stream at a fraction of the
  // device's bandwidth (8192 sites at d = 64: 4 ms per iteration with 64
  // workgroups, against about 0.4 ms for the full-device launches)
  if (nrhs > 2 || g.V > 2048) return false;
  const int Gmax = coarsest_groups(g.V);
  const size_t coef_bytes = 2 * 2 * sizeof(double) * (size_t)nrhs * (m + 2);
  if (coef_bytes > 65536) return false;
  if (coarsest_ws_doubles(nrhs, m, Gmax) > dws_cap || coarsest_ws_ints(nrhs) > iws_cap) return false;
  CoopGmres a;
  a.g = g;
  a.nrhs = nrhs;
  a.m = m;
  a.reltol = reltol;
  CoopGmresWs ws;
  ws.V = Vbasis;
  ws.w = w;
  double* p = dws;
  ws.part1 = p; p += 2 * (size_t)Gmax * nrhs * (m + 2);
  ws.part2 = p; p += 2 * (size_t)Gmax * nrhs * (m + 2);
  ws.R = p; p += 2 * (size_t)nrhs * m * m;
  ws.cs = p; p += 2 * (size_t)nrhs * m;
  ws.sn = p; p += (size_t)nrhs * m;
  ws.gv = p; p += 2 * (size_t)nrhs * (m + 1);
  ws.tolabs = p; p += nrhs;
  ws.bar = reinterpret_cast<unsigned*>(iws);
  ws.err = iws + 2;
  ws.stat = iws + 3;
  ws.flags = iws + 8;
  ws.kdone = iws + 8 + nrhs;
  hipError_t e;
  switch (d) {
    case 24: e = gmres_launch<T, S, 24>(a, coef_bytes, Dc, b, x, mu_dev, ws, st); break;
    case 32: e = gmres_launch<T, S, 32>(a, coef_bytes, Dc, b, x, mu_dev, ws, st); break;
    case 48: e = gmres_launch<T, S, 48>(a, coef_bytes, Dc, b, x, mu_dev, ws, st); break;
    default: e = gmres_launch<T, S, 64>(a, coef_bytes, Dc, b, x, mu_dev, ws, st); break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

#define INST_COOP(T, S)                                                                                             \
  template bool launch_coarse_apply_site<T, S>(const CoarseGeom&, int, const SP<S>*, const cplx<T>*, cplx<T>*,    \
                                               int, const double*, hipStream_t);                                  \
  template bool launch_sap_coarse_fused<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, const cplx<T>*,    \
                                              cplx<T>*, int, const double*, const int*, int, const int*, int, int,  \
                                              int, cplx<T>* const*, cplx<T>* const*, double* const*, long,          \
                                              hipStream_t);                                                         \
  template bool launch_coarsest_gmres<T, S>(const CoarseGeom&, int, const SP<S>*, const cplx<T>*, cplx<T>*, int,   \
                                            const double*, int, double, cplx<T>*, cplx<T>*, double*, size_t, int*, \
                                            size_t, hipStream_t);
INST_COOP(double, double)
INST_COOP(float, float)
INST_COOP(float, __hip_bfloat16)
INST_COOP(float, __half)
