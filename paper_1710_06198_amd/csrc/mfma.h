// bf16 matrix-core helpers: a split of FP32 values into two bf16 parts
// (v = hi + lo, hi = bf16(v), lo = bf16(v - hi): v to 2^-18 of its size)
// and the operand vectors of the 16x16x16 bf16 MFMA builtin.
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

