// Persistent cooperative kernels for the coarse levels.
//
// Coarse lattices are small (a few hundred to a few thousand sites), so a
// launch per Krylov or MR step leaves the GPU idle and a thread per matrix
// row is latency-bound.  These kernels run a whole coarse-level SAP smoother
// or a whole coarsest-level GMRES in one cooperative launch.  The unit of
// work is one coarse site (for one right-hand side): a 256-thread workgroup
// stages the nine input vectors the site needs in LDS and forms the D rows
// of D_c with every thread owning four consecutive rows and a slice of the
// 9*D-term sum (one 4-wide vector load per term), followed by an LDS
// reduction over the slices.  Global information (MR alphas, Gram-Schmidt
// coefficients, norms) is combined with wave-parallel reductions between
// grid barriers.  Every loop containing a barrier has a trip count that all
// workgroups evaluate identically.
#include <hip/hip_cooperative_groups.h>

#include "kernels.h"

namespace cg = cooperative_groups;

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

// Partial products of one site's D rows: red[ks][i] (ks < KS) summed over
// ks gives sum_{b in mask} sum_j Dm[b][j][i] vst[b*D + j].  Ends with a
// workgroup barrier.
template <int D> struct SiteMV {
  static constexpr int RG = D / 4;        // row groups of 4 rows
  static constexpr int KS = 256 / RG;     // slices of the 9*D-term sum
};
template <typename T, typename S, int D>
TM_D void site_mv(const SP<S>* __restrict__ Dm, const cplx<T>* vst, unsigned mask, cplx<T>* red) {
  constexpr int RG = SiteMV<D>::RG, KS = SiteMV<D>::KS, K = 9 * D;
  const int t = threadIdx.x, rg = t % RG, ks = t / RG;
  if (ks < KS) {
    cplx<T> a0 = mk<T>(0, 0), a1 = a0, a2 = a0, a3 = a0;
#pragma unroll 4
    for (int k = ks; k < K; k += KS) {
      const int b = k / D;
      if (!((mask >> b) & 1u)) continue;
      const Quad<S> q = *reinterpret_cast<const Quad<S>*>(Dm + (size_t)k * D + 4 * rg);
      const cplx<T> v = vst[k];
      cfma(a0, Store<S>::template cvt<T>(q.e[0]), v);
      cfma(a1, Store<S>::template cvt<T>(q.e[1]), v);
      cfma(a2, Store<S>::template cvt<T>(q.e[2]), v);
      cfma(a3, Store<S>::template cvt<T>(q.e[3]), v);
    }
    cplx<T>* o = red + ks * D + 4 * rg;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
    o[3] = a3;
  }
  __syncthreads();
}
template <typename T, int D>
TM_D cplx<T> site_mv_row(const cplx<T>* red, int i) {
  cplx<T> s = mk<T>(0, 0);
  for (int ks = 0; ks < SiteMV<D>::KS; ++ks) s += red[ks * D + i];
  return s;
}

// ------------------------------------------------------------------ SAP (whole smoother)
struct CoopSap {
  CoarseGeom g;
  CBlk cb;
  const int* bl[2];
  int nb[2];
  int sweeps, mr_steps, nrhs;
};

// k sweeps of SAP on D_c z = eta.  Unit = (block of the colour, site of the
// block, right-hand side).  Per colour: r = eta - D_c z on every block
// site; then per MR step q = D_B rho, per-unit partial dot products, a
// barrier, the block's alpha summed over its sites in a fixed order, and
// z += alpha rho, rho -= alpha q.
template <typename T, typename S, int D>
__global__ void __launch_bounds__(256) k_sap_coarse_coop(CoopSap a, const SP<S>* __restrict__ Dc,
                                                         const cplx<T>* __restrict__ eta, cplx<T>* z, cplx<T>* rho_g,
                                                         cplx<T>* q_g, double* part, const double* __restrict__ mu_dev) {
  cg::grid_group grid = cg::this_grid();
  __shared__ cplx<T> vst[9 * D];
  __shared__ cplx<T> red[SiteMV<D>::KS * D];
  __shared__ cplx<T> alpha_s;
  const CoarseGeom& g = a.g;
  const CBlk& cb = a.cb;
  const long VD = g.V * D;
  const int nbs = cb.nbs, nrhs = a.nrhs;
  const int t = threadIdx.x;
  for (int sw = 0; sw < a.sweeps; ++sw) {
    for (int col = 0; col < 2; ++col) {
      const int* bl = a.bl[col];
      const int units = a.nb[col] * nbs * nrhs;
      // residual
      for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int r = u % nrhs, tt = u / nrhs, sl = tt % nbs, bi = tt / nbs;
        C4 c, lc;
        cblk_site(cb, bl[bi], sl, c, lc);
        const long y = cc_index(g, c);
        const cplx<T>* zr = z + r * VD;
        for (int k = t; k < 9 * D; k += 256) {
          const int b = k / D, j = k - b * D;
          const long src = b == 0 ? y : cc_nbr(g, c, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
          vst[k] = zr[src * D + j];
        }
        __syncthreads();
        site_mv<T, S, D>(Dc + y * 9L * D * D, vst, 0x1FFu, red);
        if (t < D) {
          const T mu = (T)mu_dev[r];
          cplx<T> acc = site_mv_row<T, D>(red, t);
          acc += (t < D / 2 ? mu : -mu) * times_i(vst[t]);
          rho_g[r * VD + y * D + t] = eta[r * VD + y * D + t] - acc;
        }
        __syncthreads();
      }
      __threadfence();
      grid.sync();
      for (int it = 0; it < a.mr_steps; ++it) {
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
          const int r = u % nrhs, tt = u / nrhs, sl = tt % nbs, bi = tt / nbs;
          const int blk = bl[bi];
          C4 c, lc;
          cblk_site(cb, blk, sl, c, lc);
          const long y = cc_index(g, c);
          const cplx<T>* rr = rho_g + r * VD;
          unsigned mask = 1u;
          for (int b = 1; b < 9; ++b)
            if (cblk_nbr(cb, lc, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1) >= 0) mask |= 1u << b;
          for (int k = t; k < 9 * D; k += 256) {
            const int b = k / D, j = k - b * D;
            const int nl = b == 0 ? sl : cblk_nbr(cb, lc, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
            cplx<T> v = mk<T>(0, 0);
            if (nl >= 0) {
              C4 cn, lcn;
              cblk_site(cb, blk, nl, cn, lcn);
              v = rr[cc_index(g, cn) * D + j];
            }
            vst[k] = v;
          }
          __syncthreads();
          site_mv<T, S, D>(Dc + y * 9L * D * D, vst, mask, red);
          if (t < 64) {
            T qq = 0, qre = 0, qim = 0;
            if (t < D) {
              const T mu = (T)mu_dev[r];
              const cplx<T> rho = vst[t];
              cplx<T> acc = site_mv_row<T, D>(red, t);
              acc += (t < D / 2 ? mu : -mu) * times_i(rho);
              q_g[r * VD + y * D + t] = acc;
              qq = norm2(acc);
              const cplx<T> tq = cmulc(acc, rho);
              qre = tq.re;
              qim = tq.im;
            }
            qq = wave_sum(qq);
            qre = wave_sum(qre);
            qim = wave_sum(qim);
            if (t == 0) {
              part[3L * u] = qq;
              part[3L * u + 1] = qre;
              part[3L * u + 2] = qim;
            }
          }
          __syncthreads();
        }
        __threadfence();
        grid.sync();
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
          const int r = u % nrhs, tt = u / nrhs, sl = tt % nbs, bi = tt / nbs;
          if (t < 64) {
            double sq = 0, sre = 0, sim = 0;
            for (int q = t; q < nbs; q += 64) {
              const long o = 3L * (((long)bi * nbs + q) * nrhs + r);
              sq += part[o];
              sre += part[o + 1];
              sim += part[o + 2];
            }
            sq = wave_sum(sq);
            sre = wave_sum(sre);
            sim = wave_sum(sim);
            if (t == 0) alpha_s = sq > 0 ? mk<T>((T)(sre / sq), (T)(sim / sq)) : mk<T>(0, 0);
          }
          __syncthreads();
          if (t < D) {
            C4 c, lc;
            cblk_site(cb, bl[bi], sl, c, lc);
            const long o = r * VD + cc_index(g, c) * D + t;
            const cplx<T> alpha = alpha_s;
            const cplx<T> rho = rho_g[o];
            cfma(z[o], alpha, rho);
            rho_g[o] = rho - alpha * q_g[o];
          }
          __syncthreads();
        }
        __threadfence();
        grid.sync();
      }
    }
  }
}

static int max_coresident(const void* kern, int threads, size_t shmem) {
  int dev = 0, per_cu = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, shmem);
  return std::max(1, per_cu * ncu);
}

template <typename T, typename S, int D>
static hipError_t sap_coop_launch(CoopSap a, const SP<S>* Dc, const cplx<T>* eta, cplx<T>* z, cplx<T>* rho_g,
                                  cplx<T>* q_g, double* part, const double* mu_dev, hipStream_t st) {
  const void* kern = reinterpret_cast<const void*>(&k_sap_coarse_coop<T, S, D>);
  static int cap = 0;
  if (cap == 0) cap = std::min(2048, max_coresident(kern, 256, 0));
  const int units = std::max(a.nb[0], a.nb[1]) * a.cb.nbs * a.nrhs;
  dim3 grid(std::max(1, std::min(cap, units)));
  void* args[] = {&a, (void*)&Dc, (void*)&eta, (void*)&z, (void*)&rho_g, (void*)&q_g, (void*)&part, (void*)&mu_dev};
  return hipLaunchCooperativeKernel(kern, grid, dim3(256), args, 0, st);
}

// returns false when this shape has no cooperative kernel (caller falls back)
template <typename T, typename S>
bool launch_sap_coarse_coop(const CoarseGeom& g, int d, const int blk[4], const SP<S>* Dc, const cplx<T>* eta,
                            cplx<T>* z, int nrhs, const double* mu_dev, const int* bl0, int n0, const int* bl1, int n1,
                            int sweeps, int mr_steps, cplx<T>* rho_g, cplx<T>* q_g, double* part, long part_cap,
                            hipStream_t st) {
  if (!(d == 24 || d == 32 || d == 48 || d == 64)) return false;
  CoopSap a;
  a.g = g;
  a.cb.nbs = 1;
  for (int m = 0; m < 4; ++m) { a.cb.B[m] = blk[m]; a.cb.NB[m] = g.L[m] / blk[m]; a.cb.nbs *= blk[m]; }
  a.bl[0] = bl0;
  a.bl[1] = bl1;
  a.nb[0] = n0;
  a.nb[1] = n1;
  a.sweeps = sweeps;
  a.mr_steps = mr_steps;
  a.nrhs = nrhs;
  if ((long)std::max(n0, n1) * a.cb.nbs * nrhs * 3 > part_cap) return false;
  hipError_t e;
  switch (d) {
    case 24: e = sap_coop_launch<T, S, 24>(a, Dc, eta, z, rho_g, q_g, part, mu_dev, st); break;
    case 32: e = sap_coop_launch<T, S, 32>(a, Dc, eta, z, rho_g, q_g, part, mu_dev, st); break;
    case 48: e = sap_coop_launch<T, S, 48>(a, Dc, eta, z, rho_g, q_g, part, mu_dev, st); break;
    default: e = sap_coop_launch<T, S, 64>(a, Dc, eta, z, rho_g, q_g, part, mu_dev, st); break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// ------------------------------------------------------------------ coarsest GMRES
struct CoopGmres {
  CoarseGeom g;
  int nrhs, m;
  double reltol;
};

struct CoopGmresWs {
  void* V;          // [(m+1)][nrhs][n] cplx<T>
  void* w;          // [nrhs][n]
  double* part;     // [V][nrhs][m+1] complex: per-site partial sums
  double* coef;     // [nrhs][m+1] complex: reduced Gram-Schmidt coefficients
  double* nrm;      // [nrhs]
  double* H;        // [nrhs][m+1][m] complex
  double* cs;       // [nrhs][m] complex
  double* sn;       // [nrhs][m]
  double* gv;       // [nrhs][m+1] complex
  double* y;        // [nrhs][m] complex
  double* tolabs;   // [nrhs]
  int* flags;       // [nrhs]
  int* kdone;       // [nrhs]
};

// Sum the per-site partials of pair (r, i) over all sites with one wave per
// pair, pairs spread over every wave of the grid; fixed order, so every run
// gives the same bits.
TM_D void reduce_pairs(const double* part, int nsites, int nrhs, int m, int npairs, int ni, double* coef,
                       double* H, int j, int pass, bool cplx_out, double* nrm) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int q = gw; q < npairs; q += nw) {
    const int r = q / ni, i = q - r * ni;
    double sre = 0, sim = 0;
    for (int u = lane; u < nsites; u += 64) {
      const long o = 2L * (((long)u * nrhs + r) * (m + 1) + i);
      sre += part[o];
      sim += part[o + 1];
    }
    sre = wave_sum(sre);
    sim = wave_sum(sim);
    if (lane == 0) {
      if (cplx_out) {
        coef[2L * (r * (m + 1) + i)] = sre;
        coef[2L * (r * (m + 1) + i) + 1] = sim;
        double* h = H + 2L * ((long)r * (m + 1) * m + (long)i * m + j);
        if (pass == 0) { h[0] = sre; h[1] = sim; }
        else { h[0] += sre; h[1] += sim; }
      } else {
        nrm[r] = sqrt(sre);
      }
    }
  }
}

// GMRES(m) from x = 0 for D_c(mu_r) x_r = b_r, stopping a right-hand side
// when its implicit residual <= reltol * ||b_r||.  Classical Gram-Schmidt
// with one re-orthogonalisation; Givens updates by workgroup 0.
template <typename T, typename S, int D>
__global__ void __launch_bounds__(256) k_coarsest_gmres(CoopGmres a, const SP<S>* __restrict__ Dc,
                                                        const cplx<T>* __restrict__ b, cplx<T>* x,
                                                        const double* __restrict__ mu_dev, CoopGmresWs ws) {
  cg::grid_group grid = cg::this_grid();
  __shared__ cplx<T> vst[9 * D];
  __shared__ cplx<T> red[SiteMV<D>::KS * D];
  __shared__ int any_active;
  const CoarseGeom& g = a.g;
  const int nrhs = a.nrhs, m = a.m;
  const long n = g.V * D;
  const int nsites = (int)g.V;
  cplx<T>* V = static_cast<cplx<T>*>(ws.V);
  cplx<T>* w = static_cast<cplx<T>*>(ws.w);
  const long vs = (long)nrhs * n;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;

  // ||b_r||
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    if (t < 64)
      for (int r = 0; r < nrhs; ++r) {
        double s2 = t < D ? (double)norm2(b[r * n + (long)u * D + t]) : 0.0;
        s2 = wave_sum(s2);
        if (t == 0) { ws.part[2L * (((long)u * nrhs + r) * (m + 1))] = s2; ws.part[2L * (((long)u * nrhs + r) * (m + 1)) + 1] = 0; }
      }
  __threadfence();
  grid.sync();
  reduce_pairs(ws.part, nsites, nrhs, m, nrhs, 1, nullptr, nullptr, 0, 0, false, ws.nrm);
  __threadfence();
  grid.sync();
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    for (int k = t; k < nrhs * D; k += 256) {
      const int r = k / D, i = k - r * D;
      const double bt = ws.nrm[r];
      const long o = r * n + (long)u * D + i;
      V[o] = bt > 0 ? (T)(1.0 / bt) * b[o] : mk<T>(0, 0);
    }
  if (blockIdx.x == 0)
    for (int r = t; r < nrhs; r += 256) {
      const double bt = ws.nrm[r];
      for (int i = 0; i <= m; ++i) { ws.gv[2 * (r * (m + 1) + i)] = 0; ws.gv[2 * (r * (m + 1) + i) + 1] = 0; }
      ws.gv[2 * r * (m + 1)] = bt;
      ws.tolabs[r] = a.reltol * bt;
      ws.kdone[r] = 0;
      ws.flags[r] = (bt > 0 && bt < 1e300) ? 1 : 0;
    }
  __threadfence();
  grid.sync();

  for (int j = 0; j < m; ++j) {
    if (t == 0) {
      int any = 0;
      for (int r = 0; r < nrhs; ++r) any |= ws.flags[r];
      any_active = any;
    }
    __syncthreads();
    if (!any_active) break;   // identical in every workgroup: flags only change before a barrier
    const cplx<T>* vj = V + (long)j * vs;
    // w = D_c(mu) v_j, one site unit at a time
    for (int u = blockIdx.x; u < nsites; u += gridDim.x) {
      const C4 c = cc_coords(g, u);
      for (int r = 0; r < nrhs; ++r) {
        if (!ws.flags[r]) continue;   // uniform across the workgroup
        const cplx<T>* vr = vj + r * n;
        for (int k = t; k < 9 * D; k += 256) {
          const int bb = k / D, jj = k - bb * D;
          const long src = bb == 0 ? u : cc_nbr(g, c, (bb - 1) >> 1, ((bb - 1) & 1) ? -1 : 1);
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
    // two Gram-Schmidt passes: per-site partials, grid reduction, update
    for (int pass = 0; pass < 2; ++pass) {
      for (int u = blockIdx.x; u < nsites; u += gridDim.x)
        for (int q = wv; q < nrhs * (j + 1); q += 4) {
          const int r = q / (j + 1), i = q - r * (j + 1);
          double sre = 0, sim = 0;
          if (ws.flags[r] && lane < D) {
            const cplx<T> av = V[(long)i * vs + r * n + (long)u * D + lane];
            const cplx<T> cw = w[r * n + (long)u * D + lane];
            sre = (double)av.re * cw.re + (double)av.im * cw.im;
            sim = (double)av.re * cw.im - (double)av.im * cw.re;
          }
          sre = wave_sum(sre);
          sim = wave_sum(sim);
          if (lane == 0) {
            const long o = 2L * (((long)u * nrhs + r) * (m + 1) + i);
            ws.part[o] = sre;
            ws.part[o + 1] = sim;
          }
        }
      __threadfence();
      grid.sync();
      reduce_pairs(ws.part, nsites, nrhs, m, nrhs * (j + 1), j + 1, ws.coef, ws.H, j, pass, true, nullptr);
      __threadfence();
      grid.sync();
      for (int u = blockIdx.x; u < nsites; u += gridDim.x)
        for (int k = t; k < nrhs * D; k += 256) {
          const int r = k / D, i = k - r * D;
          if (!ws.flags[r]) continue;
          const long o = r * n + (long)u * D + i;
          cplx<T> acc = w[o];
          for (int l = 0; l <= j; ++l)
            cfma(acc, mk<T>((T)(-ws.coef[2L * (r * (m + 1) + l)]), (T)(-ws.coef[2L * (r * (m + 1) + l) + 1])),
                 V[(long)l * vs + o]);
          w[o] = acc;
        }
      __syncthreads();   // the next phase reads w of this workgroup's sites from other threads
    }
    // norm of w
    for (int u = blockIdx.x; u < nsites; u += gridDim.x)
      if (t < 64)
        for (int r = 0; r < nrhs; ++r) {
          double s2 = (ws.flags[r] && t < D) ? (double)norm2(w[r * n + (long)u * D + t]) : 0.0;
          s2 = wave_sum(s2);
          if (t == 0) { ws.part[2L * (((long)u * nrhs + r) * (m + 1))] = s2; ws.part[2L * (((long)u * nrhs + r) * (m + 1)) + 1] = 0; }
        }
    __threadfence();
    grid.sync();
    reduce_pairs(ws.part, nsites, nrhs, m, nrhs, 1, nullptr, nullptr, 0, 0, false, ws.nrm);
    __threadfence();
    grid.sync();
    cplx<T>* vn = V + (long)(j + 1) * vs;
    for (int u = blockIdx.x; u < nsites; u += gridDim.x)
      for (int k = t; k < nrhs * D; k += 256) {
        const int r = k / D, i = k - r * D;
        const double hn = ws.nrm[r];
        const long o = r * n + (long)u * D + i;
        vn[o] = hn > 0 ? (T)(1.0 / hn) * w[o] : mk<T>(0, 0);
      }
    __syncthreads();
    if (blockIdx.x == 0)
      for (int r = t; r < nrhs; r += 256) {
        if (!ws.flags[r]) continue;
        double* H = ws.H + 2L * r * (m + 1) * m;
        double* cs = ws.cs + 2L * r * m;
        double* sn = ws.sn + (long)r * m;
        double* gg = ws.gv + 2L * r * (m + 1);
        const double hn = ws.nrm[r];
        // previous rotations [[c, s], [-s, conj(c)]] (s real) on column j
        double ar = H[2 * j], ai = H[2 * j + 1];
        for (int i = 0; i < j; ++i) {
          const double br = H[2 * ((i + 1) * m + j)], bi = H[2 * ((i + 1) * m + j) + 1];
          const double cr = cs[2 * i], ci = cs[2 * i + 1], s = sn[i];
          H[2 * (i * m + j)] = cr * ar - ci * ai + s * br;
          H[2 * (i * m + j) + 1] = cr * ai + ci * ar + s * bi;
          const double ur = -s * ar + (cr * br + ci * bi);
          const double ui = -s * ai + (cr * bi - ci * br);
          ar = ur;
          ai = ui;
        }
        const double den = sqrt(ar * ar + ai * ai + hn * hn);
        if (!(den > 0) || den != den) { ws.flags[r] = 0; continue; }
        const double cr = ar / den, ci = -ai / den, s = hn / den;
        cs[2 * j] = cr;
        cs[2 * j + 1] = ci;
        sn[j] = s;
        H[2 * (j * m + j)] = den;
        H[2 * (j * m + j) + 1] = 0;
        const double gr = gg[2 * j], gi = gg[2 * j + 1];
        gg[2 * (j + 1)] = -s * gr;
        gg[2 * (j + 1) + 1] = -s * gi;
        gg[2 * j] = cr * gr - ci * gi;
        gg[2 * j + 1] = cr * gi + ci * gr;
        ws.kdone[r] = j + 1;
        const double res = s * sqrt(gr * gr + gi * gi);
        if (res <= ws.tolabs[r] || hn <= 1e-15 * den || j + 1 >= m) ws.flags[r] = 0;
      }
    __threadfence();
    grid.sync();
  }
  // y = R^-1 g, then x = V y
  if (blockIdx.x == 0)
    for (int r = t; r < nrhs; r += 256) {
      const int k = ws.kdone[r];
      const double* H = ws.H + 2L * r * (m + 1) * m;
      const double* gg = ws.gv + 2L * r * (m + 1);
      double* yv = ws.y + 2L * r * m;
      for (int i = k - 1; i >= 0; --i) {
        double sr = gg[2 * i], si = gg[2 * i + 1];
        for (int l = i + 1; l < k; ++l) {
          const double hr = H[2 * (i * m + l)], hi = H[2 * (i * m + l) + 1];
          sr -= hr * yv[2 * l] - hi * yv[2 * l + 1];
          si -= hr * yv[2 * l + 1] + hi * yv[2 * l];
        }
        const double dr = H[2 * (i * m + i)], di = H[2 * (i * m + i) + 1];
        const double dd = dr * dr + di * di;
        yv[2 * i] = (sr * dr + si * di) / dd;
        yv[2 * i + 1] = (si * dr - sr * di) / dd;
      }
    }
  __threadfence();
  grid.sync();
  for (int u = blockIdx.x; u < nsites; u += gridDim.x)
    for (int k = t; k < nrhs * D; k += 256) {
      const int r = k / D, i = k - r * D;
      const int kd = ws.kdone[r];
      const double* yv = ws.y + 2L * r * m;
      const long o = r * n + (long)u * D + i;
      cplx<T> acc = mk<T>(0, 0);
      for (int l = 0; l < kd; ++l) cfma(acc, mk<T>((T)yv[2 * l], (T)yv[2 * l + 1]), V[(long)l * vs + o]);
      x[o] = acc;
    }
}

template <typename T, typename S, int D>
static hipError_t gmres_coop_launch(CoopGmres a, const SP<S>* Dc, const cplx<T>* b, cplx<T>* x, const double* mu_dev,
                                    CoopGmresWs ws, hipStream_t st) {
  const void* kern = reinterpret_cast<const void*>(&k_coarsest_gmres<T, S, D>);
  static int cap = 0;
  if (cap == 0) cap = std::min(2048, max_coresident(kern, 256, 0));
  const int G = (int)std::max<long>(1, std::min<long>(cap, a.g.V));
  void* args[] = {&a, (void*)&Dc, (void*)&b, (void*)&x, (void*)&mu_dev, &ws};
  return hipLaunchCooperativeKernel(kern, dim3(G), dim3(256), args, 0, st);
}

size_t coarsest_ws_doubles(long n, int nrhs, int m, int nsites) {
  (void)n;
  return 2 * (size_t)nsites * nrhs * (m + 1) + (size_t)nrhs * (2 * (m + 1) + 1 + 2 * (m + 1) * m + 2 * m + m +
                                                              2 * (m + 1) + 2 * m + 1);
}

template <typename T, typename S>
bool launch_coarsest_gmres(const CoarseGeom& g, int d, const SP<S>* Dc, const cplx<T>* b, cplx<T>* x, int nrhs,
                           const double* mu_dev, int m, double reltol, cplx<T>* Vbasis, cplx<T>* w, double* dws,
                           size_t dws_cap, int* iws, hipStream_t st) {
  if (!(d == 24 || d == 32 || d == 48 || d == 64)) return false;
  if (coarsest_ws_doubles(g.V * d, nrhs, m, (int)g.V) > dws_cap) return false;
  CoopGmres a;
  a.g = g;
  a.nrhs = nrhs;
  a.m = m;
  a.reltol = reltol;
  CoopGmresWs ws;
  ws.V = Vbasis;
  ws.w = w;
  double* p = dws;
  ws.part = p; p += 2 * (size_t)g.V * nrhs * (m + 1);
  ws.coef = p; p += 2 * (size_t)nrhs * (m + 1);
  ws.nrm = p; p += nrhs;
  ws.H = p; p += 2 * (size_t)nrhs * (m + 1) * m;
  ws.cs = p; p += 2 * (size_t)nrhs * m;
  ws.sn = p; p += (size_t)nrhs * m;
  ws.gv = p; p += 2 * (size_t)nrhs * (m + 1);
  ws.y = p; p += 2 * (size_t)nrhs * m;
  ws.tolabs = p; p += nrhs;
  ws.flags = iws;
  ws.kdone = iws + nrhs;
  hipError_t e;
  switch (d) {
    case 24: e = gmres_coop_launch<T, S, 24>(a, Dc, b, x, mu_dev, ws, st); break;
    case 32: e = gmres_coop_launch<T, S, 32>(a, Dc, b, x, mu_dev, ws, st); break;
    case 48: e = gmres_coop_launch<T, S, 48>(a, Dc, b, x, mu_dev, ws, st); break;
    default: e = gmres_coop_launch<T, S, 64>(a, Dc, b, x, mu_dev, ws, st); break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

#define INST_COOP(T, S)                                                                                             \
  template bool launch_sap_coarse_coop<T, S>(const CoarseGeom&, int, const int*, const SP<S>*, const cplx<T>*,     \
                                             cplx<T>*, int, const double*, const int*, int, const int*, int, int,   \
                                             int, cplx<T>*, cplx<T>*, double*, long, hipStream_t);                 \
  template bool launch_coarsest_gmres<T, S>(const CoarseGeom&, int, const SP<S>*, const cplx<T>*, cplx<T>*, int,   \
                                            const double*, int, double, cplx<T>*, cplx<T>*, double*, size_t, int*, \
                                            hipStream_t);
INST_COOP(double, double)
INST_COOP(float, float)
INST_COOP(float, __hip_bfloat16)
INST_COOP(float, __half)
