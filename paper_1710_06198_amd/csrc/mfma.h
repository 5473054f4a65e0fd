// bf16 matrix-core helpers: a split of FP32 values into two bf16 parts
// (v = hi + lo, hi = bf16(v), lo = bf16(v - hi): v to 2^-18 of its size)
// and the complex tile products on gfx950's 16x16x32 bf16 MFMA.
#pragma once

#include "common.h"

typedef short mf_s4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
TM_D unsigned short bf16_bits_rne(float x) {   // round to nearest even
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
TM_D float bf16_bits_float(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

struct MfSplit {
  mf_s4 rh, rl, ih, il, nih, nil, nrh, nrl;   // hi/lo parts of Re v, Im v, -Im v and -Re v
};
TM_D MfSplit mf_split(const cplx<float>* v) {
  MfSplit o;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const unsigned short rh = bf16_bits_rne(v[e].re), ih = bf16_bits_rne(v[e].im);
    const unsigned short rl = bf16_bits_rne(v[e].re - bf16_bits_float(rh));
    const unsigned short il = bf16_bits_rne(v[e].im - bf16_bits_float(ih));
    o.rh[e] = (short)rh;
    o.rl[e] = (short)rl;
    o.ih[e] = (short)ih;
    o.il[e] = (short)il;
    o.nih[e] = (short)(ih ^ 0x8000u);
    o.nil[e] = (short)(il ^ 0x8000u);
    o.nrh[e] = (short)(rh ^ 0x8000u);
    o.nrl[e] = (short)(rl ^ 0x8000u);
  }
  return o;
}


// The complex products of one 16x16 tile over 16 values of k on the
// 16x16x32 bf16 MFMA (lane l: rows / columns l % 16 of A / B, the eight
// values 8 (l / 16) + e of the k axis; C as for the 16x16x16 form: rows
// 4 (l / 16) + v, column l % 16, checked on the GPU with exact small
// integers).  The eight k slots of a lane carry the real parts (e < 4) and
// the imaginary parts (e >= 4) of A's four entries, so one instruction
// takes both halves of a complex multiply-add:
//   mf_cmac:       accr += Re(A v), acci += Im(A v)
//   mf_cmac_conj:  accr += Re(conj(A) v), acci += Im(conj(A) v)
// for A = ar + i ai (exact in bf16) and v split into hi and lo parts: four
// instructions per tile where the 16x16x16 form takes eight.
typedef short mf_s8 __attribute__((ext_vector_type(8)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));
TM_D mf_s8 mf_cat(mf_s4 a, mf_s4 b) {
  mf_s8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = a[e];
    r[4 + e] = b[e];
  }
  return r;
}
TM_D mf_f4 mf_mma32(mf_s8 a, mf_s8 b, mf_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mf_bf8, a), __builtin_bit_cast(mf_bf8, b), c, 0,
                                                 0, 0);
}
TM_D void mf_cmac(mf_s4 ar, mf_s4 ai, const MfSplit& bb, mf_f4& accr, mf_f4& acci) {
  const mf_s8 a = mf_cat(ar, ai);
  accr = mf_mma32(a, mf_cat(bb.rh, bb.nih), accr);
  accr = mf_mma32(a, mf_cat(bb.rl, bb.nil), accr);
  acci = mf_mma32(a, mf_cat(bb.ih, bb.rh), acci);
  acci = mf_mma32(a, mf_cat(bb.il, bb.rl), acci);
}
TM_D void mf_cmac_conj(mf_s4 ar, mf_s4 ai, const MfSplit& bb, mf_f4& accr, mf_f4& acci) {
  const mf_s8 a = mf_cat(ar, ai);
  accr = mf_mma32(a, mf_cat(bb.rh, bb.ih), accr);
  accr = mf_mma32(a, mf_cat(bb.rl, bb.il), accr);
  acci = mf_mma32(a, mf_cat(bb.ih, bb.nrh), acci);
  acci = mf_mma32(a, mf_cat(bb.il, bb.nrl), acci);
}
