// Device helpers shared by the batched MFMA surface kernels: packed FP16
// complex arithmetic in MFMA operand layouts, the FP16 hi / remainder split of
// an FP32 value, and wave reductions of the window peak (top value, its
// position, runner-up) with DPP inside 16-lane rows.
#pragma once

#include "internal.h"

namespace ca {

constexpr int MF_RSRC_WORD3 = 0x00020000;  // raw buffer descriptor, 32-bit data format

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// The arrays of a clip set the kernel reads (a compact kernel argument).
struct MfView {
  const __half2* spec16;
  const int64_t* spec_off;
  const uint64_t* bits;
  const int64_t* bits_off;
  const int32_t* npix;
  const int16_t* w;
  const int32_t* zero_bins;
};

__host__ inline MfView mf_view(const ClipsDev& c) {
  return MfView{c.spec16, c.spec_off, c.bits, c.bits_off, c.npix, c.w, c.zero_bins};
}

__device__ __forceinline__ h2_t as_h2(uint32_t x) { return __builtin_bit_cast(h2_t, x); }
__device__ __forceinline__ uint32_t as_u32(h2_t x) { return __builtin_bit_cast(uint32_t, x); }

// -i z on a packed FP16 (re, im) pair: (im, -re) in one packed multiply by
// 1.0 whose operand selects swap the halves and negate the new high half
// (the compiler otherwise spends a swap and a sign flip).
__device__ __forceinline__ h2_t mul_neg_i(h2_t z) {
  uint32_t r;
  asm("v_pk_mul_f16 %0, %1, 1.0 op_sel:[1,0] op_sel_hi:[0,0] neg_hi:[1,0]" : "=v"(r) : "v"(as_u32(z)));
  return as_h2(r);
}

// m * conj(r) on packed FP16 (re, im) pairs.
__device__ __forceinline__ h2_t cmulc_h2(h2_t m, h2_t r) {
  const h2_t rr = {r.x, r.x};
  const h2_t ri = {r.y, -r.y};
  const h2_t ms = {m.y, m.x};
  return m * rr + ms * ri;
}

// Two FP32 values as FP16 pairs: their truncation (hi, one packing
// instruction) and the remainder lo = value - hi rounded to nearest.  One
// mixed-precision FMA per value forms value - hi exactly (the two are close)
// and rounds it into its half of lo, so the pair carries the value to about
// 2^-22.
__device__ __forceinline__ void split_f16(float a, float b, h2_t& hi, h2_t& lo) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
  hi = __builtin_bit_cast(h2_t, h);
  uint32_t l;
  asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=&v"(l) : "v"(h), "v"(a));
  asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(l) : "v"(h), "v"(b));
  lo = __builtin_bit_cast(h2_t, l);
}

// s times the low / high FP16 half of z, as FP32, in one mixed-precision
// multiply-add each (the conversion is exact).
__device__ __forceinline__ float sgn_lo(h2_t z, float s) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, 0 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(as_u32(z)), "v"(s));
  return r;
}
__device__ __forceinline__ float sgn_hi(h2_t z, float s) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, 0 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(as_u32(z)), "v"(s));
  return r;
}

// A wave-uniform 64-bit value from lane l.
__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Cross-lane reads for wave reductions: DPP within 16-lane rows (quad
// permutes, half-row and row mirrors).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, x)));
}

// Merge a top-two state with another lane's: larger value wins, ties to the
// lower position; commutative, so both lanes of a swap end up equal.
__device__ __forceinline__ void top2_merge(float& v1, int& i1, float& v2, float o1, int oi, float o2) {
  const bool take = o1 > v1 || (o1 == v1 && oi < i1);
  const float a = take ? v1 : o1;  // the loser's top
  const float b = take ? o2 : v2;  // the winner's runner-up
  v2 = a > b ? a : b;
  v1 = take ? o1 : v1;
  i1 = take ? oi : i1;
}

template <int CTRL>
__device__ __forceinline__ void top2_step(float& v1, int& i1, float& v2) {
  top2_merge(v1, i1, v2, dpp_f<CTRL>(v1), dpp_i<CTRL>(i1), dpp_f<CTRL>(v2));
}

// Top value, its position and the runner-up over the wave (positions break
// ties low): DPP steps reduce each 16-lane row, then the four row results are
// read as wave-uniform values and merged.
__device__ __forceinline__ void wave_top2(float& v1, int& i1, float& v2) {
  top2_step<0xB1>(v1, i1, v2);   // quad_perm [1,0,3,2]
  top2_step<0x4E>(v1, i1, v2);   // quad_perm [2,3,0,1]
  top2_step<0x141>(v1, i1, v2);  // row_half_mirror
  top2_step<0x140>(v1, i1, v2);  // row_mirror
  auto rd = [&](int l, float& a1, int& ai, float& a2) {
    a1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v1), l));
    ai = __builtin_amdgcn_readlane(i1, l);
    a2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v2), l));
  };
  float r1, r2, o1, o2;
  int ri, oi;
  rd(0, r1, ri, r2);
  rd(16, o1, oi, o2);
  top2_merge(r1, ri, r2, o1, oi, o2);
  rd(32, o1, oi, o2);
  top2_merge(r1, ri, r2, o1, oi, o2);
  rd(48, o1, oi, o2);
  top2_merge(r1, ri, r2, o1, oi, o2);
  v1 = r1;
  i1 = ri;
  v2 = r2;
}

// Sum over the wave (wave-uniform result).
__device__ __forceinline__ int wave_sum(int c) {
  c += dpp_i<0xB1>(c);
  c += dpp_i<0x4E>(c);
  c += dpp_i<0x141>(c);
  c += dpp_i<0x140>(c);
  return __builtin_amdgcn_readlane(c, 0) + __builtin_amdgcn_readlane(c, 16) + __builtin_amdgcn_readlane(c, 32) +
         __builtin_amdgcn_readlane(c, 48);
}

}  // namespace ca
