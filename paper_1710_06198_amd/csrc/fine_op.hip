// Fine-level kernels: layout conversion, clover build, the twisted-mass
// clover Wilson stencil and the SAP block solver.
//
// D(mu) psi(x) = A(x) psi(x) + i mu g5 psi(x)
//   - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)]
// (twisted-mass term of Sec. 1.1 on the clover-improved Wilson operator).
#include "fine_site.h"

// ------------------------------------------------------------------ conversion
__global__ void k_convert_links(FineGeom g, const cplx<double>* __restrict__ canon, cplx<double>* out64,
                                cplx<float>* out32, int antiperiodic) {
  long cs = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (cs >= g.V) return;
  int mu = blockIdx.y;
  int c[4];
  long r = cs;
  c[0] = (int)(r % g.L[0]); r /= g.L[0];
  c[1] = (int)(r % g.L[1]); r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
  long s = fine_index(g, c);
  double sign = (antiperiodic && mu == 3 && c[3] == g.L[3] - 1) ? -1.0 : 1.0;
  const cplx<double>* src = canon + ((long)mu * g.V + cs) * 9;
  const size_t ob = (size_t)mu * 9 * g.V + tsite((unsigned)s, 9);
  for (int k = 0; k < 9; ++k) {
    cplx<double> v = sign * src[k];
    size_t o = ob + k * FT;
    if (out64) out64[o] = v;
    if (out32) out32[o] = mk<float>((float)v.re, (float)v.im);
  }
}

void launch_convert_links(const FineGeom& g, const cplx<double>* canon, cplx<double>* out64, cplx<float>* out32,
                          int antiperiodic, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), 4);
  hipLaunchKernelGGL(k_convert_links, grid, dim3(256), 0, st, g, canon, out64, out32, antiperiodic);
}

template <typename T>
__global__ void k_spinor_to_internal(FineGeom g, const cplx<double>* __restrict__ canon, cplx<T>* __restrict__ out) {
  long cs = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (cs >= g.V) return;
  long rhs = blockIdx.y;
  int c[4];
  long r = cs;
  c[0] = (int)(r % g.L[0]); r /= g.L[0];
  c[1] = (int)(r % g.L[1]); r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
  long s = fine_index(g, c);
  const cplx<double>* src = canon + (rhs * g.V + cs) * 12;
  cplx<T>* dst = out + rhs * 12 * g.V + tsite((unsigned)s, 12);
  for (int k = 0; k < 12; ++k) dst[k * FT] = mk<T>((T)src[k].re, (T)src[k].im);
}

template <typename T>
__global__ void k_spinor_to_canonical(FineGeom g, const cplx<T>* __restrict__ in, cplx<double>* __restrict__ canon) {
  long cs = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (cs >= g.V) return;
  long rhs = blockIdx.y;
  int c[4];
  long r = cs;
  c[0] = (int)(r % g.L[0]); r /= g.L[0];
  c[1] = (int)(r % g.L[1]); r /= g.L[1];
  c[2] = (int)(r % g.L[2]);
  c[3] = (int)(r / g.L[2]);
  long s = fine_index(g, c);
  const cplx<T>* src = in + rhs * 12 * g.V + tsite((unsigned)s, 12);
  cplx<double>* dst = canon + (rhs * g.V + cs) * 12;
  for (int k = 0; k < 12; ++k) {
    cplx<T> v = src[k * FT];
    dst[k] = mk<double>((double)v.re, (double)v.im);
  }
}

template <typename T>
void launch_spinor_to_internal(const FineGeom& g, const cplx<double>* canon, cplx<T>* out, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_to_internal<T>, grid, dim3(256), 0, st, g, canon, out);
}
template <typename T>
void launch_spinor_to_canonical(const FineGeom& g, const cplx<T>* in, cplx<double>* canon, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_to_canonical<T>, grid, dim3(256), 0, st, g, in, canon);
}
template void launch_spinor_to_internal<double>(const FineGeom&, const cplx<double>*, cplx<double>*, int, hipStream_t);
template void launch_spinor_to_internal<float>(const FineGeom&, const cplx<double>*, cplx<float>*, int, hipStream_t);
template void launch_spinor_to_canonical<double>(const FineGeom&, const cplx<double>*, cplx<double>*, int, hipStream_t);
template void launch_spinor_to_canonical<float>(const FineGeom&, const cplx<float>*, cplx<double>*, int, hipStream_t);

// ------------------------------------------------------------------ clover (K2)
__device__ long shifted_site(const FineGeom& g, const int c[4], int m1, int s1, int m2, int s2) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  if (s1) cc[m1] = (cc[m1] + s1 + g.L[m1]) % g.L[m1];
  if (s2) cc[m2] = (cc[m2] + s2 + g.L[m2]) % g.L[m2];
  return fine_index(g, cc);
}

// Q_{mu nu}(x) = sum of the four same-orientation plaquette leaves at x;
// Fhat = (Q - Q^dag)/8 with its trace removed; A_s = (m0+4) + sum_{mu<nu}
// [c_sw (i/2) sigma_{mu nu}]_s (x) Fhat_{mu nu}.
__global__ void k_clover_build(FineGeom g, const cplx<double>* __restrict__ U, CloverCoef cc, double* clov64,
                               float* clov32) {
  long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  fine_coords(g, s, c);
  cplx<double> A[2][6][6];
  for (int ch = 0; ch < 2; ++ch)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) A[ch][i][j] = mk(i == j ? cc.diag : 0.0, 0.0);
  int p = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++p) {
      long x = s;
      long xpm = shifted_site(g, c, mu, 1, nu, 0);
      long xpn = shifted_site(g, c, nu, 1, mu, 0);
      long xmm = shifted_site(g, c, mu, -1, nu, 0);
      long xmn = shifted_site(g, c, nu, -1, mu, 0);
      long xmmpn = shifted_site(g, c, mu, -1, nu, 1);
      long xpmmn = shifted_site(g, c, mu, 1, nu, -1);
      long xmmmn = shifted_site(g, c, mu, -1, nu, -1);
      M3<double> Um_x = load_link(U, mu, x, g.V), Un_x = load_link(U, nu, x, g.V);
      M3<double> Un_xpm = load_link(U, nu, xpm, g.V), Um_xpn = load_link(U, mu, xpn, g.V);
      M3<double> Um_xmm = load_link(U, mu, xmm, g.V), Un_xmm = load_link(U, nu, xmm, g.V);
      M3<double> Um_xmmpn = load_link(U, mu, xmmpn, g.V);
      M3<double> Um_xmmmn = load_link(U, mu, xmmmn, g.V), Un_xmmmn = load_link(U, nu, xmmmn, g.V);
      M3<double> Un_xmn = load_link(U, nu, xmn, g.V), Um_xmn = load_link(U, mu, xmn, g.V);
      M3<double> Un_xpmmn = load_link(U, nu, xpmmn, g.V);
      // l1 = Um(x) Un(x+mu) Um(x+nu)^dag Un(x)^dag
      M3<double> l1 = m3_mul_ad(m3_mul_ad(m3_mul(Um_x, Un_xpm), Um_xpn), Un_x);
      // l2 = Un(x) Um(x-mu+nu)^dag Un(x-mu)^dag Um(x-mu)
      M3<double> l2 = m3_mul(m3_mul_ad(m3_mul_ad(Un_x, Um_xmmpn), Un_xmm), Um_xmm);
      // l3 = Um(x-mu)^dag Un(x-mu-nu)^dag Um(x-mu-nu) Un(x-nu)
      M3<double> l3 = m3_mul(m3_mul(m3_mul_da(Um_xmm, m3_dag(Un_xmmmn)), Um_xmmmn), Un_xmn);
      // l4 = Un(x-nu)^dag Um(x-nu) Un(x+mu-nu) Um(x)^dag
      M3<double> l4 = m3_mul_ad(m3_mul(m3_mul_da(Un_xmn, Um_xmn), Un_xpmmn), Um_x);
      M3<double> q = m3_add(m3_add(l1, l2), m3_add(l3, l4));
      cplx<double> F[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i][j] = 0.125 * (q.e[i][j] - conj(q.e[j][i]));
      cplx<double> tr = (1.0 / 3.0) * (F[0][0] + F[1][1] + F[2][2]);
      for (int i = 0; i < 3; ++i) F[i][i] -= tr;
      for (int ch = 0; ch < 2; ++ch)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            cplx<double> sg = mk(cc.re[p][ch][a][b], cc.im[p][ch][a][b]);
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) A[ch][a * 3 + i][b * 3 + j] += sg * F[i][j];
          }
    }
  for (int ch = 0; ch < 2; ++ch) {
    const size_t base = (size_t)ch * 36 * g.V + tsite((unsigned)s, 36);
    for (int i = 0; i < 6; ++i) {
      double v = A[ch][i][i].re;
      if (clov64) clov64[base + i * FT] = v;
      if (clov32) clov32[base + i * FT] = (float)v;
    }
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        const size_t k = 6 + 2 * herm_idx(i, j);
        cplx<double> v = A[ch][i][j];
        if (clov64) { clov64[base + k * FT] = v.re; clov64[base + (k + 1) * FT] = v.im; }
        if (clov32) { clov32[base + k * FT] = (float)v.re; clov32[base + (k + 1) * FT] = (float)v.im; }
      }
  }
}

void launch_clover_build(const FineGeom& g, const cplx<double>* links64, const CloverCoef& cc, double* clov64,
                         float* clov32, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_build, dim3((unsigned)((g.V + 127) / 128)), dim3(128), 0, st, g, links64, cc, clov64,
                     clov32);
}


// ------------------------------------------------------------------ stencil
// One workgroup per block (one thread per site).  The block's spinors are
// staged in LDS once; hops that stay in the block read them there.  The
// backward hop is formed by its source: site y computes
// U_mu(y)^dag (1 + g_mu) psi(y) as a half spinor with the link it already
// loaded for its forward hop and leaves it in LDS for y + mu, so every
// link of the block is read once.  Only hops across the block surface read
// the neighbouring block's spinor (and, backwards, its link) from memory;
// in FP32 those of the x and y faces are read at the start of the block,
// next to the neighbouring blocks' own loads (all four directions would
// need LDS for three more faces and cost a workgroup per CU).
// Workgroups are mapped so that each XCD sweeps a contiguous range of
// blocks, keeping neighbouring blocks' faces in the same L2.
// Index of a site of the block on the face normal to MU: its local index
// with the MU coordinate removed.
template <int MU>
TM_D int face_index(const FineGeom& g, int loc) {
  const int ls = g.lstride[MU];
  return loc % ls + (loc / (ls * g.B[MU])) * ls;
}

// Surface hops of direction MU loaded at the start of the block: a site on
// the forward face keeps (1 - g_mu) psi(x + mu) projected, a site on the
// backward face U_mu(x - mu)^dag (1 + g_mu) psi(x - mu), as half spinors in
// LDS (ff, fb: [6][face sites]).  Neighbouring blocks on the same XCD start
// within a few microseconds of each other and load these spinors at their
// own start too, so the two reads of each line meet in L2.
template <int MU, typename T>
TM_D void load_faces(const FineOp<T>& op, const cplx<T>* __restrict__ in, unsigned s, int loc, const int c[4],
                     cplx<T>* ff, cplx<T>* fb) {
  const FineGeom& g = op.g;
  if (g.NB[MU] == 1) return;
  const int B = g.B[MU], lc = c[MU] % B, fsz = g.bvol / B, fi = face_index<MU>(g, loc);
  if (lc == B - 1) {
    cplx<T> pn[12], h[6];
    load_spinor(in, (unsigned)fine_neighbour(g, s, c, MU, +1), g.V, pn);
    project<MU, -1>(pn, h);
#pragma unroll
    for (int k = 0; k < 6; ++k) ff[k * fsz + fi] = h[k];
  } else if (lc == 0) {
    cplx<T> pn[12], h[6], w[6];
    const unsigned sb = (unsigned)fine_neighbour(g, s, c, MU, -1);
    load_spinor(in, sb, g.V, pn);
    const M3<T> ub = load_link_u<MU>(op.links, sb, g.V);
    project<MU, +1>(pn, h);
    su3_dmv(ub, h, w);
    su3_dmv(ub, h + 3, w + 3);
#pragma unroll
    for (int k = 0; k < 6; ++k) fb[k * fsz + fi] = w[k];
  }
}

template <int MU, bool STREAM, typename T>
TM_D void stage_dir(const FineOp<T>& op, const cplx<T>* __restrict__ in, const cplx<T>* psl, cplx<T>* hb, unsigned s,
                    int loc, const int c[4], const cplx<T>* psi, cplx<T>* acc, const cplx<T>* ff = nullptr,
                    const cplx<T>* fb = nullptr) {
  const FineGeom& g = op.g;
  const long V = g.V;
  const int bv = g.bvol, ls = g.lstride[MU], B = g.B[MU];
  const int lc = c[MU] % B;
  const bool whole = g.NB[MU] == 1;
  const M3<T> u = STREAM ? load_link_stream<MU>(op.links, s, V) : load_link_u<MU>(op.links, s, V);
  {
    // half spinor sent to y + mu: U^dag (1 + g) psi
    cplx<T> h[6], w[6];
    project<MU, +1>(psi, h);
    su3_dmv(u, h, w);
    su3_dmv(u, h + 3, w + 3);
#pragma unroll
    for (int k = 0; k < 6; ++k) hb[k * bv + loc] = w[k];
  }
  {
    cplx<T> pn[12];
    const int nl = lc < B - 1 ? loc + ls : (whole ? loc - (B - 1) * ls : -1);
    if (nl >= 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) pn[k] = psl[k * bv + nl];
      hop_fwd<MU>(u, pn, acc);
    } else if (ff) {
      const int fsz = bv / B, fi = face_index<MU>(g, loc);
      cplx<T> h[6], w[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = ff[k * fsz + fi];
      su3_mv(u, h, w);
      su3_mv(u, h + 3, w + 3);
      reconstruct<MU, -1>(w, acc);
    } else {
      load_spinor(in, (unsigned)fine_neighbour(g, s, c, MU, +1), V, pn);
      hop_fwd<MU>(u, pn, acc);
    }
  }
  compiler_fence(acc);
  __syncthreads();
  {
    const int nl = lc > 0 ? loc - ls : (whole ? loc + (B - 1) * ls : -1);
    if (nl >= 0 || fb) {
      const cplx<T>* src = nl >= 0 ? hb + nl : fb + face_index<MU>(g, loc);
      const int str = nl >= 0 ? bv : bv / B;
      cplx<T> w[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) w[k] = src[k * str];
      reconstruct<MU, +1>(w, acc);
    } else {
      cplx<T> pn[12];
      const unsigned sb = (unsigned)fine_neighbour(g, s, c, MU, -1);
      load_spinor(in, sb, V, pn);
      const M3<T> ub = load_link_u<MU>(op.links, sb, V);
      hop_bwd<MU>(ub, pn, acc);
    }
  }
  compiler_fence(acc);
  __syncthreads();   // hb is overwritten by the next direction
}

template <typename T, bool STREAM>
TM_D void dslash_block_rhs(const FineOp<T>& op, const cplx<T>* __restrict__ inr, cplx<T>* __restrict__ outr, T mu,
                           cplx<T>* psl, cplx<T>* hb, unsigned s, int loc, const int c[4]) {
  const long V = op.g.V;
  const int bv = op.g.bvol;
  cplx<T> psi[12], acc[12];
  load_spinor(inr, s, V, psi);
#pragma unroll
  for (int k = 0; k < 12; ++k) psl[k * bv + loc] = psi[k];
  // FP32: the x and y surface hops are loaded up front (LDS after hb)
  constexpr bool EARLY = sizeof(T) == 4;
  cplx<T>* ff0 = hb + 6 * bv;
  cplx<T>* fb0 = ff0 + 6 * (bv / op.g.B[0]);
  cplx<T>* ff1 = fb0 + 6 * (bv / op.g.B[0]);
  cplx<T>* fb1 = ff1 + 6 * (bv / op.g.B[1]);
  if constexpr (EARLY) {
    load_faces<0>(op, inr, s, loc, c, ff0, fb0);
    load_faces<1>(op, inr, s, loc, c, ff1, fb1);
  }
  site_diag<T, STREAM>(op, s, mu, psi, acc);
  compiler_fence(acc);
  __syncthreads();
  const bool w0 = op.g.NB[0] == 1, w1 = op.g.NB[1] == 1;
  stage_dir<0, STREAM>(op, inr, psl, hb, s, loc, c, psi, acc, EARLY && !w0 ? ff0 : nullptr,
                       EARLY && !w0 ? fb0 : nullptr);
  stage_dir<1, STREAM>(op, inr, psl, hb, s, loc, c, psi, acc, EARLY && !w1 ? ff1 : nullptr,
                       EARLY && !w1 ? fb1 : nullptr);
  stage_dir<2, STREAM>(op, inr, psl, hb, s, loc, c, psi, acc);
  stage_dir<3, STREAM>(op, inr, psl, hb, s, loc, c, psi, acc);
  // the output is written non-temporally: its lines would otherwise take
  // L2 from the neighbouring blocks' face spinors (32^3 x 64: one RHS
  // 0.375 -> 0.351 ms, 12 RHS 3.16 -> 3.10 ms)
  cplx<T>* o = outr + tsite(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) st_stream(o + k * FT, acc[k]);
}

// A single right-hand side streams links and clover (non-temporal loads).
// A batch gives each (block, right-hand side) pair its own workgroup, the
// right-hand sides of one block back to back on one XCD, so the block's
// links and clover come from that L2 after the first (a loop over the
// right-hand sides inside one workgroup kept the links in registers,
// 211 VGPRs, half the occupancy).
template <typename T, bool BATCH>
__global__ void __launch_bounds__(256) k_dslash(FineOp<T> op, const cplx<T>* __restrict__ in,
                                                cplx<T>* __restrict__ out, const double* __restrict__ mu_dev,
                                                int nrhs) {
  extern __shared__ unsigned char smem_raw[];
  const FineGeom& g = op.g;
  const long V = g.V;
  const int bv = g.bvol;
  cplx<T>* psl = reinterpret_cast<cplx<T>*>(smem_raw);   // [12][bv]
  cplx<T>* hb = psl + 12 * bv;                          // [6][bv]
  // XCD x (= blockIdx.x % 8) takes blocks [x * per, (x + 1) * per), and in a
  // batch each of them nrhs times in a row
  const int per = (g.nblocks + 7) / 8;
  const int rest = (int)(blockIdx.x >> 3);
  const int r = BATCH ? rest % nrhs : 0;
  const int blk = (int)(blockIdx.x & 7) * per + (BATCH ? rest / nrhs : rest);
  if (blk >= g.nblocks) return;
  const int loc = threadIdx.x;
  const unsigned s = (unsigned)blk * bv + loc;
  int c[4];
  fine_coords(g, s, c);
  dslash_block_rhs<T, !BATCH>(op, in + (long)r * 12 * V, out + (long)r * 12 * V, (T)mu_dev[r], psl, hb, s, loc, c);
}

template <typename T>
void launch_dslash(const FineOp<T>& op, const cplx<T>* in, cplx<T>* out, int nrhs, const double* mu_dev,
                   hipStream_t st) {
  const int per = (op.g.nblocks + 7) / 8;
  size_t lds = 18 * (size_t)op.g.bvol * sizeof(cplx<T>);
  if (sizeof(T) == 4) lds += 12 * (size_t)(op.g.bvol / op.g.B[0] + op.g.bvol / op.g.B[1]) * sizeof(cplx<T>);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_dslash<T, false>), dim3((unsigned)(8 * per)), dim3(op.g.bvol), lds, st, op, in, out, mu_dev,
                       nrhs);
  else
    hipLaunchKernelGGL((k_dslash<T, true>), dim3((unsigned)(8 * per * nrhs)), dim3(op.g.bvol), lds, st, op, in, out,
                       mu_dev, nrhs);
}
template void launch_dslash<double>(const FineOp<double>&, const cplx<double>*, cplx<double>*, int, const double*,
                                    hipStream_t);
template void launch_dslash<float>(const FineOp<float>&, const cplx<float>*, cplx<float>*, int, const double*,
                                   hipStream_t);

template <typename T>
__global__ void k_gamma5_fine(long V, const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out) {
  unsigned s = blockIdx.x * 256u + threadIdx.x;
  if (s >= V) return;
  size_t base = (size_t)blockIdx.y * 12 * V + tsite(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    cplx<T> v = in[base + k * FT];
    out[base + k * FT] = k < 6 ? v : -v;
  }
}
template <typename T>
void launch_gamma5_fine(const FineGeom& g, const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_gamma5_fine<T>, grid, dim3(256), 0, st, g.V, in, out);
}
template void launch_gamma5_fine<double>(const FineGeom&, const cplx<double>*, cplx<double>*, int, hipStream_t);
template void launch_gamma5_fine<float>(const FineGeom&, const cplx<float>*, cplx<float>*, int, hipStream_t);

// ------------------------------------------------------------------ SAP (K3)
template <typename T, int MINB, int BV>
__global__ void __launch_bounds__(256, MINB) k_sap_fine(FineOp<T> op, const cplx<T>* __restrict__ eta, cplx<T>* z,
                                                  const double* __restrict__ mu_dev, const int* __restrict__ blist,
                                                  int nblk, int nrhs, int mr_steps) {
  sap_block_solve<T, MINB, false, false, BV>(op, eta, z, mu_dev, blist, nblk, nrhs, mr_steps);
}

template <typename T>
void launch_sap_fine(const FineOp<T>& op, const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu_dev,
                     const int* block_list, int nblk, int mr_steps, hipStream_t st, double epsbar) {
  const size_t red_bytes = 2 * 6 * 8 * sizeof(T);   // two slots of [waves <= 8][halves][3]
  const size_t sh = (size_t)12 * op.g.bvol * sizeof(cplx<T>) + red_bytes;
  const unsigned n8 = (unsigned)((nblk + 7) / 8 * 8);
  if constexpr (sizeof(T) == 4) {
    const int tv = tune_get(TUNE_SAP0, op.g.bvol, op.g.V, nrhs);
    const bool coupled = epsbar != 0.0 && nrhs == 2 && op.g.bvol % 32 == 0;
    if (coupled || (tv == 2 && op.g.bvol % 32 == 0)) {
      // two right-hand sides per workgroup, the MR vectors of both in LDS
      const size_t sh2 = sh + (size_t)12 * op.g.bvol * sizeof(cplx<T>);
      launch_sap_fine_pair(op, eta, z, nrhs, mu_dev, block_list, nblk, mr_steps, sh2, n8, st,
                           coupled ? epsbar : 0.0);
      if (coupled) return;
      tune_used(TUNE_SAP0, 2);
      return;
    }
    if (tv >= 0 ? tv == 1 : nrhs > 1) {
      const size_t sh3 = sh + (size_t)12 * op.g.bvol * sizeof(cplx<T>);   // and e
      // 4^4 blocks: the block volume as a constant turns the LDS addresses
      // of the 12 components into immediate offsets of one base
      if (op.g.bvol == 256)
        hipLaunchKernelGGL((k_sap_fine<T, 3, 256>), dim3(n8 * nrhs), dim3(op.g.bvol), sh3, st, op, eta, z, mu_dev,
                           block_list, nblk, nrhs, mr_steps);
      else
        hipLaunchKernelGGL((k_sap_fine<T, 3, 0>), dim3(n8 * nrhs), dim3(op.g.bvol), sh3, st, op, eta, z, mu_dev,
                           block_list, nblk, nrhs, mr_steps);
      tune_used(TUNE_SAP0, 1);
      return;
    }
  }
  tune_used(TUNE_SAP0, 0);
  if (op.g.bvol == 256)
    hipLaunchKernelGGL((k_sap_fine<T, 1, 256>), dim3(n8 * nrhs), dim3(op.g.bvol), sh, st, op, eta, z, mu_dev,
                       block_list, nblk, nrhs, mr_steps);
  else
    hipLaunchKernelGGL((k_sap_fine<T, 1, 0>), dim3(n8 * nrhs), dim3(op.g.bvol), sh, st, op, eta, z, mu_dev,
                       block_list, nblk, nrhs, mr_steps);
}
template void launch_sap_fine<double>(const FineOp<double>&, const cplx<double>*, cplx<double>*, int, const double*,
                                      const int*, int, int, hipStream_t, double);
template void launch_sap_fine<float>(const FineOp<float>&, const cplx<float>*, cplx<float>*, int, const double*,
                                     const int*, int, int, hipStream_t, double);

// ------------------------------------------------------------------ even-odd reduction
// v_r = 0 on the sites of parity `par` (x + y + z + t), per right-hand side
template <typename T>
__global__ void k_zero_parity(FineGeom g, cplx<T>* v, int par) {
  const unsigned s = blockIdx.x * 256u + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  fine_coords(g, s, c);
  if (((c[0] + c[1] + c[2] + c[3]) & 1) != par) return;
  cplx<T>* o = v + (long)blockIdx.y * 12 * g.V + tsite(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k * FT] = mk<T>(0, 0);
}
template <typename T>
void launch_zero_parity(const FineGeom& g, cplx<T>* v, int nrhs, int parity, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_parity<T>, dim3((unsigned)((g.V + 255) / 256), nrhs), dim3(256), 0, st, g, v, parity);
}
template void launch_zero_parity<double>(const FineGeom&, cplx<double>*, int, int, hipStream_t);

// D_hat(mu) = D_ee - D_eo D_oo^-1 D_oe on the even sites (x + y + z + t even):
// the hopping term only joins opposite parities and A + i mu g5 is
// site-diagonal.  Two gather passes over one parity each: on the odd sites
// t = (A + i mu g5)^-1 sum_hops(psi), on the even sites
// out = (A + i mu g5) psi - sum_hops(t); odd outputs are 0.

// y = (A_ch + i s mu)^-1 v for one chirality block of a site (s = +1 for
// the upper spins, -1 for the lower): Gaussian elimination without pivoting,
// stable because the Hermitian part A_ch is positive definite whenever
// m0 + 4 exceeds the spectral radius of the clover term (every workload here).
template <typename T>
TM_D void clover_block_solve(const T* __restrict__ cl, unsigned s, T smu, const cplx<T>* v, cplx<T>* y) {
  cplx<T> a[6][6], b[6];
  const T* p = cl + tsite(s, 36);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    a[i][i] = mk<T>(p[i * FT], smu);
    b[i] = v[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      const int k = 6 + 2 * herm_idx(i, j);
      a[i][j] = mk<T>(p[k * FT], p[(k + 1) * FT]);
      a[j][i] = conj(a[i][j]);
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T d = (T)1 / norm2(a[k][k]);
    const cplx<T> inv = d * conj(a[k][k]);
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      const cplx<T> f = a[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < 6; ++j) a[i][j] -= f * a[k][j];
      b[i] -= f * b[k];
    }
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    cplx<T> t = b[i];
#pragma unroll
    for (int j = i + 1; j < 6; ++j) t -= a[i][j] * y[j];
    const T d = (T)1 / norm2(a[i][i]);
    y[i] = t * (d * conj(a[i][i]));
  }
}

// PAR = 1: t = D_oo^-1 D_oe psi on the odd sites (and out = 0 there); PAR = 0:
// out = D_ee psi - D_eo t on the even sites.  One thread per site of the
// lattice, all right-hand sides along y; threads on the other parity only
// exit.  (Packing one parity into consecutive threads halves the idle
// lanes but makes every lane's loads stride-2 in the tiled layout, which
// measured slower: 0.42 against 0.37 ms on 24^3 x 48.)
template <typename T, int PAR>
__global__ void __launch_bounds__(256) k_schur_half(FineOp<T> op, const cplx<T>* __restrict__ psi,
                                                    cplx<T>* __restrict__ t, cplx<T>* __restrict__ out,
                                                    const double* __restrict__ mu_dev) {
  const long V = op.g.V;
  const unsigned s = blockIdx.x * 256u + threadIdx.x;
  if (s >= V) return;
  int c[4];
  fine_coords(op.g, s, c);
  if (((c[0] + c[1] + c[2] + c[3]) & 1) != PAR) return;
  const int r = blockIdx.y;
  const T mu = (T)mu_dev[r];
  const cplx<T>* pr = psi + (long)r * 12 * V;
  cplx<T>* o = out + (long)r * 12 * V + tsite(s, 12);
  const cplx<T>* src = PAR == 1 ? pr : t + (long)r * 12 * V;   // t: odd sites only
  cplx<T> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<T>(0, 0);
  site_hops_dir<0>(op, src, s, c, acc);
  compiler_fence(acc);
  site_hops_dir<1>(op, src, s, c, acc);
  compiler_fence(acc);
  site_hops_dir<2>(op, src, s, c, acc);
  compiler_fence(acc);
  site_hops_dir<3>(op, src, s, c, acc);
  compiler_fence(acc);
  if constexpr (PAR == 1) {
    cplx<T> y[12];
    clover_block_solve(op.clover, s, mu, acc, y);
    clover_block_solve(op.clover + 36 * V, s, -mu, acc + 6, y + 6);
    cplx<T>* tt = t + (long)r * 12 * V + tsite(s, 12);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      tt[k * FT] = y[k];
      o[k * FT] = mk<T>(0, 0);
    }
  } else {
    cplx<T> p[12], d[12];
    load_spinor(pr, s, V, p);
    site_diag(op, s, mu, p, d);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k * FT] = d[k] - acc[k];
  }
}

template <typename T>
void launch_schur(const FineOp<T>& op, const cplx<T>* in, cplx<T>* tmp, cplx<T>* out, int nrhs, const double* mu_dev,
                  hipStream_t st) {
  const dim3 grid((unsigned)((op.g.V + 255) / 256), (unsigned)nrhs);
  hipLaunchKernelGGL((k_schur_half<T, 1>), grid, dim3(256), 0, st, op, in, tmp, out, mu_dev);
  hipLaunchKernelGGL((k_schur_half<T, 0>), grid, dim3(256), 0, st, op, in, tmp, out, mu_dev);
}
template void launch_schur<double>(const FineOp<double>&, const cplx<double>*, cplx<double>*, cplx<double>*, int,
                                   const double*, hipStream_t);
template void launch_schur<float>(const FineOp<float>&, const cplx<float>*, cplx<float>*, cplx<float>*, int,
                                  const double*, hipStream_t);
