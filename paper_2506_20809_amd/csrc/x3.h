// Three-piece bf16 matrix-core products of FP32 operands and the lane
// exchanges they are reduced with; shared by the far-field pair kernels and
// the tree far field.
#pragma once

#include <hip/hip_runtime.h>

namespace sbie {

using f4 = float __attribute__((ext_vector_type(4)));
using u4 = unsigned __attribute__((ext_vector_type(4)));
using bf8 = __bf16 __attribute__((ext_vector_type(8)));

// Three-piece bf16 form.  An FP32 value x splits exactly into bf16 pieces
// x = x_h + x_m + x_l of 8 significant bits each (round to nearest, then twice
// on the remainder).  Lane group k of a 16x16x32 bf16 product owns eight K
// slots; term k of a K = 4 contraction a.b takes six of them,
//     a_h b_h + a_h b_m + a_m b_h + a_h b_l + a_l b_h + a_m b_m,
// which is a_k b_k less a_m b_l + a_l b_m + a_l b_l (relative size 2^-24 and
// below).  In registers, two bf16 per dword (low half first):
//     A = (a_h a_h) (a_m a_h) (a_l a_m) (s6 s7)
//     B = (b_h b_m) (b_h b_l) (b_h b_m) (t6 t7).
// The last two slots add one exact FP32 value e per column (the accumulator
// input of the FP32 form): lane groups 0 and 1 of B hold (e_h e_m) and (e_l 0)
// against (1 1) and (1 0) in A, the other groups zeros.  Every product is exact
// in FP32 and the matrix core sums them in FP32.
__device__ inline unsigned bf16_bits(__bf16 h) { return (unsigned)__builtin_bit_cast(unsigned short, h); }

__device__ inline void split3(float x, unsigned& h, unsigned& m, unsigned& l) {
  const __bf16 bh = (__bf16)x;
  const float r = x - (float)bh;
  const __bf16 bm = (__bf16)r;
  const __bf16 bl = (__bf16)(r - (float)bm);
  h = bf16_bits(bh);
  m = bf16_bits(bm);
  l = bf16_bits(bl);
}

// A operand of lane group lg; with `extra` the last slots take the column's e
__device__ inline u4 split_a(float x, int lg, bool extra) {
  unsigned h, m, l;
  split3(x, h, m, l);
  const unsigned s = !extra ? 0u : (lg == 0 ? 0x3F803F80u : (lg == 1 ? 0x00003F80u : 0u));
  return u4{h | h << 16, m | h << 16, l | m << 16, s};
}

// B operand of lane group lg for the value x, with the column's exact extra term e
__device__ inline u4 split_b(float x, int lg, float e) {
  unsigned h, m, l, eh, em, el;
  split3(x, h, m, l);
  split3(e, eh, em, el);
  const unsigned t = lg == 0 ? (eh | em << 16) : (lg == 1 ? el : 0u);
  return u4{h | m << 16, h | l << 16, h | m << 16, t};
}

// B operands of all four lane groups of one column: the terms x[k] and the
// column's extra term e (split once), out[k] for lane group k
__device__ inline void split_b_column(const float (&x)[4], float e, u4 (&out)[4]) {
  unsigned eh, em, el;
  split3(e, eh, em, el);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    unsigned h, m, l;
    split3(x[k], h, m, l);
    const unsigned t = k == 0 ? (eh | em << 16) : (k == 1 ? el : 0u);
    out[k] = u4{h | m << 16, h | l << 16, h | m << 16, t};
  }
}

// the FP32 value of a B operand's main term
__device__ inline float join_b(u4 v) {
  const float h = __builtin_bit_cast(float, v.x << 16);
  const float m = __builtin_bit_cast(float, v.x & 0xFFFF0000u);
  const float l = __builtin_bit_cast(float, v.y & 0xFFFF0000u);
  return (h + m) + l;
}

// v from the lane whose byte address (lane index times 4) is addr
__device__ inline float lane_value(float v, int addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ inline double lane_value(double v, int addr) {
  const int2 p = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_ds_bpermute(addr, p.x), __builtin_amdgcn_ds_bpermute(addr, p.y)));
}

// v[k] summed over the 16 lanes of each row group (lanes l with the same
// l/16), lane l keeping the sum for element l%16: recursive halving, in which
// lanes l and l^d (d = 8, 4, 2, 1) each keep one half of the remaining
// elements and add the partner's copy of that half.  The first two halvings
// add in FP32 (each result then holds two roundings), the last two in FP64.
template <int D, typename T>
__device__ inline void halve(T (&v)[16], int lane) {
  const bool hi = (lane & D) != 0;
  const int addr = (lane ^ D) << 2;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const T send = hi ? v[k] : v[D + k];
    const T keep = hi ? v[D + k] : v[k];
    v[k] = keep + lane_value(send, addr);
  }
}

__device__ inline double row_group_sums(float (&v)[16], int lane) {
  halve<8>(v, lane);
  halve<4>(v, lane);
  double w[16];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (double)v[k];
  halve<2>(w, lane);
  halve<1>(w, lane);
  return w[0];
}

// Workgroups are dispatched round-robin over the eight XCDs (w mod 8).  Each
// XCD gets a contiguous range of the work index instead, so that the
// particles it holds at once are neighbours in index and share most of their
// partners' source blocks in its L2.
__device__ inline int xcd_work_index() {
  const int G = (int)gridDim.x, w = (int)blockIdx.x;
  const int xcd = w % 8, per = G / 8, extra = G % 8;
  return xcd * per + (xcd < extra ? xcd : extra) + w / 8;
}

// one K = 4 product of three-piece operands (accumulator input in the extra slots)
__device__ inline f4 mma_x3(u4 a, u4 b) {
  const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), zero, 0, 0, 0);
}

}  // namespace sbie
