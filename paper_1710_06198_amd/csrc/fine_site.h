// Per-site pieces of the fine operator and the SAP block solve, shared by
// the translation units that instantiate the stencil and SAP kernels (the
// two-right-hand-side SAP kernel is compiled on its own: in one unit with
// the others the compiler's register allocation of those degraded).
#pragma once

#include "kernels.h"
#include "su3.h"

// ------------------------------------------------------------------ stencil
// Every access goes through a wave-uniform base (field + component * V) and
// the lane's 32-bit site index.
template <typename T>
TM_D void load_spinor(const cplx<T>* __restrict__ f, unsigned s, long V, cplx<T>* p) {
  const cplx<T>* q = f + tsite(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = q[k * FT];
}

// acc = (A + i mu g5) psi
template <typename T, bool STREAM = false>
TM_D void site_diag(const FineOp<T>& op, unsigned s, T mu, const cplx<T>* psi, cplx<T>* acc) {
  const long V = op.g.V;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<T>(0, 0);
  clover_block_mv<T, STREAM>(op.clover, s, V, psi, acc);
  clover_block_mv<T, STREAM>(op.clover + 36 * V, s, V, psi + 6, acc + 6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    acc[k] += mu * times_i(psi[k]);
    acc[6 + k] -= mu * times_i(psi[6 + k]);
  }
}

// Both hops of direction MU, gathered from memory (used where one direction
// at a time keeps the register count down)
template <int MU, typename T>
TM_D void site_hops_dir(const FineOp<T>& op, const cplx<T>* __restrict__ in, unsigned s, const int c[4],
                        cplx<T>* acc) {
  const long V = op.g.V;
  cplx<T> pn[12];
  const unsigned sf = (unsigned)fine_neighbour(op.g, s, c, MU, +1);
  load_spinor(in, sf, V, pn);
  M3<T> u = load_link_u<MU>(op.links, s, V);
  hop_fwd<MU>(u, pn, acc);
  compiler_fence(acc);
  const unsigned sb = (unsigned)fine_neighbour(op.g, s, c, MU, -1);
  load_spinor(in, sb, V, pn);
  M3<T> ub = load_link_u<MU>(op.links, sb, V);
  hop_bwd<MU>(ub, pn, acc);
}

// One hop's operands gathered from memory: the neighbouring spinor and the
// link.  Hop H is direction H / 2, forward for even H, backward for odd.
template <typename T>
struct HopRegs {
  cplx<T> p[12];
  M3<T> u;
};
template <int H, typename T>
TM_D void gather_hop(const FineOp<T>& op, const cplx<T>* __restrict__ in, unsigned s, const int c[4],
                     HopRegs<T>& r) {
  constexpr int MU = H >> 1;
  const long V = op.g.V;
  if constexpr ((H & 1) == 0) {
    load_spinor(in, (unsigned)fine_neighbour(op.g, s, c, MU, +1), V, r.p);
    r.u = load_link_u<MU>(op.links, s, V);
  } else {
    const unsigned sb = (unsigned)fine_neighbour(op.g, s, c, MU, -1);
    load_spinor(in, sb, V, r.p);
    r.u = load_link_u<MU>(op.links, sb, V);
  }
}
template <int H, typename T>
TM_D void apply_hop(const HopRegs<T>& r, cplx<T>* acc) {
  if constexpr ((H & 1) == 0) hop_fwd<(H >> 1)>(r.u, r.p, acc);
  else hop_bwd<(H >> 1)>(r.u, r.p, acc);
}
TM_D void memory_fence_compiler() { __asm__ __volatile__("" ::: "memory"); }

// Two hops of the gather in flight: the loads of hop H + 1 are issued before
// the arithmetic of hop H (register sets a and b alternate).
template <int H, typename T>
TM_D void hops_pipelined(const FineOp<T>& op, const cplx<T>* __restrict__ in, unsigned s, const int c[4],
                         HopRegs<T>& a, HopRegs<T>& b, cplx<T>* acc) {
  if constexpr (H < 7) {
    gather_hop<H + 1>(op, in, s, c, b);
    memory_fence_compiler();
    apply_hop<H>(a, acc);
    compiler_fence(acc);
    hops_pipelined<H + 1>(op, in, s, c, b, a, acc);
  } else {
    apply_hop<H>(a, acc);
  }
}

// (D(mu) in)(s) for one right-hand side, the gather pipelined (hops first,
// then the clover and twisted-mass term on the site's own value); own
// receives in(s)
template <typename T>
TM_D void site_dslash_pipelined(const FineOp<T>& op, const cplx<T>* __restrict__ in, unsigned s, T mu,
                                cplx<T>* acc, cplx<T>* own) {
  int c[4];
  fine_coords(op.g, s, c);
  const long V = op.g.V;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<T>(0, 0);
  HopRegs<T> a, b;
  gather_hop<0>(op, in, s, c, a);
  memory_fence_compiler();
  hops_pipelined<0>(op, in, s, c, a, b, acc);
  compiler_fence(acc);
  load_spinor(in, s, V, own);
  clover_block_mv<T>(op.clover, s, V, own, acc);
  clover_block_mv<T>(op.clover + 36 * V, s, V, own + 6, acc + 6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    acc[k] += mu * times_i(own[k]);
    acc[6 + k] -= mu * times_i(own[6 + k]);
  }
}

// ------------------------------------------------------------------ SAP (K3)
// One workgroup per SAP block (one thread per site).  For every block B of
// the given colour: r_B = eta_B - (D z)_B, then mr_steps of minimal residual
// on the block-restricted operator D_B (hops leaving B dropped) from e = 0,
// then z_B += e.  Blocks of one colour only neighbour blocks of the other
// colour, so blocks of one launch never read what another writes.
template <int MU, typename T, int BV = 0>
TM_D void block_hops_dir(const FineOp<T>& op, const cplx<T>* lds, unsigned s, int loc, const int c[4], cplx<T>* acc) {
  const FineGeom& g = op.g;
  const int bv = BV ? BV : g.bvol;
  const int lc = c[MU] % g.B[MU];
  const bool whole = g.NB[MU] == 1;    // block spans the periodic direction
  cplx<T> pn[12];
  // forward neighbour
  int nl = -1;
  if (lc < g.B[MU] - 1) nl = loc + g.lstride[MU];
  else if (whole) nl = loc - (g.B[MU] - 1) * g.lstride[MU];
  if (nl >= 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) pn[k] = lds[k * bv + nl];
    M3<T> u = load_link_u<MU>(op.links, (unsigned)s, g.V);
    hop_fwd<MU>(u, pn, acc);
  }
  compiler_fence(acc);
  nl = -1;
  if (lc > 0) nl = loc - g.lstride[MU];
  else if (whole) nl = loc + (g.B[MU] - 1) * g.lstride[MU];
  if (nl >= 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) pn[k] = lds[k * bv + nl];
    const unsigned sb = (unsigned)(s - loc + nl);
    M3<T> ub = load_link_u<MU>(op.links, sb, g.V);
    hop_bwd<MU>(ub, pn, acc);
  }
}

// In-block neighbour of hop H (direction H / 2, forward for even H) as a
// block-local index, or -1 where the hop leaves the block.
template <int H>
TM_D int block_nbr(const FineGeom& g, int loc, const int c[4]) {
  constexpr int MU = H >> 1;
  const int lc = c[MU] % g.B[MU];
  const bool whole = g.NB[MU] == 1;    // block spans the periodic direction
  if constexpr ((H & 1) == 0) {
    if (lc < g.B[MU] - 1) return loc + g.lstride[MU];
    return whole ? loc - (g.B[MU] - 1) * g.lstride[MU] : -1;
  } else {
    if (lc > 0) return loc - g.lstride[MU];
    return whole ? loc + (g.B[MU] - 1) * g.lstride[MU] : -1;
  }
}

// Hop H of the block residual's gather: the neighbour's value from the
// block's staged copy in LDS where the neighbour is in the block, from
// memory where it is not; the link from memory.
template <int H, typename T, int BV = 0>
TM_D void gather_hop_block(const FineOp<T>& op, const cplx<T>* __restrict__ in, const cplx<T>* zl, unsigned s,
                           int loc, const int c[4], HopRegs<T>& r) {
  constexpr int MU = H >> 1;
  const long V = op.g.V;
  const int bv = BV ? BV : op.g.bvol;
  const int nl = block_nbr<H>(op.g, loc, c);
  const unsigned sn = (unsigned)fine_neighbour(op.g, s, c, MU, (H & 1) ? -1 : +1);
  if (nl >= 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) r.p[k] = zl[k * bv + nl];
  } else {
    load_spinor(in, sn, V, r.p);
  }
  r.u = load_link_u<MU>(op.links, (H & 1) ? sn : s, V);
}
template <int H, typename T, int BV = 0>
TM_D void block_hops_pipelined(const FineOp<T>& op, const cplx<T>* __restrict__ in, const cplx<T>* zl, unsigned s,
                               int loc, const int c[4], HopRegs<T>& a, HopRegs<T>& b, cplx<T>* acc) {
  if constexpr (H < 7) {
    gather_hop_block<H + 1, T, BV>(op, in, zl, s, loc, c, b);
    memory_fence_compiler();
    apply_hop<H>(a, acc);
    compiler_fence(acc);
    block_hops_pipelined<H + 1, T, BV>(op, in, zl, s, loc, c, b, a, acc);
  } else {
    apply_hop<H>(a, acc);
  }
}

// (D(mu) z)(s) for a site of a block whose own values zl[k * bvol + loc]
// are staged in LDS (the workgroup has passed a barrier since): in-block
// neighbours from LDS, the others and the links from memory, two hops in
// flight; then the clover and twisted-mass term on the site's own value.
template <typename T, int BV = 0>
TM_D void block_site_dslash(const FineOp<T>& op, const cplx<T>* __restrict__ in, const cplx<T>* zl, unsigned s,
                            int loc, const int c[4], T mu, cplx<T>* acc) {
  const long V = op.g.V;
  const int bv = BV ? BV : op.g.bvol;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<T>(0, 0);
  HopRegs<T> a, b;
  gather_hop_block<0, T, BV>(op, in, zl, s, loc, c, a);
  memory_fence_compiler();
  block_hops_pipelined<0, T, BV>(op, in, zl, s, loc, c, a, b, acc);
  compiler_fence(acc);
  cplx<T> own[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) own[k] = zl[k * bv + loc];
  clover_block_mv<T>(op.clover, s, V, own, acc);
  clover_block_mv<T>(op.clover + 36 * V, s, V, own + 6, acc + 6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    acc[k] += mu * times_i(own[k]);
    acc[6 + k] -= mu * times_i(own[6 + k]);
  }
}

// Workgroup sums of three values, one barrier: the wave sums go to slot
// `slot` of red (two slots of 3 x 8 values).  Alternate the slot between
// calls: a slot is written again only two calls later, after every wave
// has passed the barrier that follows its reads of it.
template <typename T>
TM_D void block_reduce3(T& a, T& b, T& c, T* red, int slot) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  T* r = red + slot * 24;   // up to 8 waves
  if (lane == 0) { r[w * 3] = a; r[w * 3 + 1] = b; r[w * 3 + 2] = c; }
  __syncthreads();
  a = 0; b = 0; c = 0;
  for (int i = 0; i < nw; ++i) { a += r[i * 3]; b += r[i * 3 + 1]; c += r[i * 3 + 2]; }
}

// Sums of three values over each half-wave (lanes 0-31, 32-63), one barrier;
// red holds two slots of [waves][2 halves][3] (see block_reduce3).
template <typename T>
TM_D void block_reduce3_halves(T& a, T& b, T& c, T* red, int slot) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, half = lane >> 5, nw = blockDim.x >> 6;
  T* r = red + slot * 6 * nw;
  if ((lane & 31) == 0) { r[(w * 2 + half) * 3] = a; r[(w * 2 + half) * 3 + 1] = b; r[(w * 2 + half) * 3 + 2] = c; }
  __syncthreads();
  a = 0; b = 0; c = 0;
  for (int i = 0; i < nw; ++i) {
    a += r[(i * 2 + half) * 3];
    b += r[(i * 2 + half) * 3 + 1];
    c += r[(i * 2 + half) * 3 + 2];
  }
}

// MINB: workgroups per CU the register allocation aims for (3 for
// batches, where more resident blocks hide more of the L2 latency).
// PAIR: two right-hand sides per workgroup, 2 x bvol threads: each wave
// holds 32 sites (one layout tile) for both, lanes l and l + 32 on the
// same site, so every link and clover load of the wave covers both
// right-hand sides with the cache lines of one.
// CPL (with PAIR): the pair is the two flavours of a doublet (Sec. 1.1,
// Eq. (2)) and the block operator carries the flavour coupling: each
// flavour's D_B(+-mubar) plus -epsbar times the other flavour at the same
// site, one MR step on both flavours together (one alpha from sums over
// both halves).
template <typename T, int MINB, bool PAIR, bool CPL = false, int BV = 0>
TM_D void sap_block_solve(const FineOp<T>& op, const cplx<T>* __restrict__ eta, cplx<T>* z,
                          const double* __restrict__ mu_dev, const int* __restrict__ blist, int nblk, int nrhs,
                          int mr_steps, T epsbar = 0) {
  static_assert(!CPL || PAIR, "the flavour coupling needs both flavours in the workgroup");
  extern __shared__ unsigned char smem_raw[];
  const FineGeom& g = op.g;
  const long V = g.V;
  const int bv = BV ? BV : g.bvol;
  // batches (MINB 3): the block solution e lives in LDS next to the MR
  // vector, each thread touching only its own site (no barrier), which
  // frees the 24 registers that otherwise spill at three workgroups per CU
  constexpr bool ELDS = MINB == 3 && !PAIR;
  const int half = PAIR ? (threadIdx.x >> 5) & 1 : 0;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw) + half * 12 * bv;
  cplx<T>* el = lds + 12 * bv;
  T* red = reinterpret_cast<T*>(reinterpret_cast<cplx<T>*>(smem_raw) + (ELDS || PAIR ? 24 : 12) * bv);
  // workgroup -> (block, rhs or pair): the right-hand sides of one block
  // run on one XCD one after the other, so its links and clover come from
  // that L2 after the first; with one right-hand side this is the identity
  const int nunit = PAIR ? (nrhs + 1) / 2 : nrhs;
  const int x8 = blockIdx.x & 7, rest = blockIdx.x >> 3;
  const int ru = rest % nunit, bi = (rest / nunit) * 8 + x8;
  if (bi >= nblk) return;
  // a lone last right-hand side of a pair is computed by both halves and
  // written by the first
  const bool writes = !PAIR || 2 * ru + half < nrhs;
  const int r = PAIR ? (writes ? 2 * ru + half : 2 * ru) : ru;
  const T mu = (T)mu_dev[r];
  const int loc = PAIR ? ((threadIdx.x >> 6) << 5) | (threadIdx.x & 31) : threadIdx.x;
  const unsigned s = (unsigned)blist[bi] * bv + loc;
  const cplx<T>* zr = z + (long)r * 12 * V;
  int c[4];
  fine_coords(g, s, c);
  // e accumulates the block's new iterate from z's own value (the final
  // write needs no second read of z)
  cplx<T> rho[12], q[12], e[ELDS ? 1 : 12];
  // one RHS in FP32: the block's own z is staged in LDS (the MR vector's
  // slot, free until the first step) and the residual's in-block
  // neighbours are read from there (at the batches' register budget this
  // form spills)
  constexpr bool LDS_RESIDUAL = MINB == 1 && !PAIR && sizeof(T) == 4;
  {
    cplx<T> dz[12], zs[12];
    if constexpr (LDS_RESIDUAL) {
      load_spinor(zr, s, V, zs);
#pragma unroll
      for (int k = 0; k < 12; ++k) lds[k * bv + loc] = zs[k];
      __syncthreads();
      block_site_dslash<T, BV>(op, zr, lds, s, loc, c, mu, dz);
    } else {
      site_dslash_pipelined(op, zr, s, mu, dz, zs);
    }
    if constexpr (CPL) {
      const cplx<T>* zo = z + (long)(r ^ 1) * 12 * V + tsite(s, 12);
#pragma unroll
      for (int k = 0; k < 12; ++k) dz[k] -= epsbar * zo[k * FT];
    }
    const cplx<T>* er = eta + (long)r * 12 * V + tsite(s, 12);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      rho[k] = er[k * FT] - dz[k];
      if constexpr (ELDS) el[k * bv + loc] = zs[k];
      else if constexpr (LDS_RESIDUAL) e[k] = lds[k * bv + loc];
      else e[k] = zs[k];
    }
    // every neighbour read of the staged z is done before the first MR
    // step overwrites it
    if constexpr (LDS_RESIDUAL) __syncthreads();
  }
  for (int it = 0; it < mr_steps; ++it) {
#pragma unroll
    for (int k = 0; k < 12; ++k) lds[k * bv + loc] = rho[k];
    __syncthreads();
    site_diag(op, s, mu, rho, q);
    compiler_fence(q);
    block_hops_dir<0, T, BV>(op, lds, s, loc, c, q);
    compiler_fence(q);
    block_hops_dir<1, T, BV>(op, lds, s, loc, c, q);
    compiler_fence(q);
    block_hops_dir<2, T, BV>(op, lds, s, loc, c, q);
    compiler_fence(q);
    block_hops_dir<3, T, BV>(op, lds, s, loc, c, q);
    if constexpr (CPL) {
      // the other flavour's rho at this site, staged by the other half
      const cplx<T>* lo = reinterpret_cast<cplx<T>*>(smem_raw) + (half ^ 1) * 12 * bv;
#pragma unroll
      for (int k = 0; k < 12; ++k) q[k] -= epsbar * lo[k * bv + loc];
    }
    T qq = 0, qr_re = 0, qr_im = 0;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      acc_norm2(qq, q[k]);
      acc_dotc(qr_re, qr_im, q[k], rho[k]);
    }
    // the next step overwrites the staged rho only after this barrier,
    // which every wave reaches after its last neighbour read
    if constexpr (PAIR && !CPL) block_reduce3_halves(qq, qr_re, qr_im, red, it & 1);
    else block_reduce3(qq, qr_re, qr_im, red, it & 1);
    cplx<T> alpha = qq > (T)0 ? mk(qr_re / qq, qr_im / qq) : mk<T>(0, 0);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      if constexpr (ELDS) {
        cplx<T> ek = el[k * bv + loc];
        cfma(ek, alpha, rho[k]);
        el[k * bv + loc] = ek;
      } else {
        cfma(e[k], alpha, rho[k]);
      }
      cfms(rho[k], alpha, q[k]);
    }
  }
  if (!writes) return;
  cplx<T>* zo = z + (long)r * 12 * V + tsite(s, 12);
#pragma unroll
  for (int k = 0; k < 12; ++k) zo[k * FT] = ELDS ? el[k * bv + loc] : e[k];
}

