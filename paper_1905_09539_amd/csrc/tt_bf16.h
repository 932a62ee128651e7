// Multi-term BF16 products for the low-precision recursion updates and
// transforms of mixed-precision refinement (gfx950).
//
// A float64 operand x is split into three bfloat16 terms x = h + m + l + e
// with |e| <= 2^-24 |x| (each term rounds the remainder of the previous ones
// to bfloat16; the remainders are exact in float64).  A product of two
// split operands keeps the six terms with combined order <= 2,
//   x y ~ h_x h_y + h_x m_y + m_x h_y + m_x m_y + h_x l_y + l_x h_y,
// all accumulated in FP32 by v_mfma_f32_16x16x16_bf16: FP32-level accuracy
// from BF16 matrix cores (the splitting of Henry, Tang and Heinecke,
// "Leveraging the bfloat16 artificial intelligence datatype for
// higher-precision computations", ARITH 2019).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tt {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bfloat16 bits
__device__ inline uint16_t bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline double bf16_value(uint16_t b) { return (double)__uint_as_float((uint32_t)b << 16); }

// x ~ h + m + l (bfloat16 bits)
__device__ inline void split3(double x, uint16_t& h, uint16_t& m, uint16_t& l) {
    h = bf16_bits((float)x);
    const double r1 = x - bf16_value(h);
    m = bf16_bits((float)r1);
    const double r2 = r1 - bf16_value(m);
    l = bf16_bits((float)r2);
}

// Split operands of one 16x16x16 step: lane holds four K values of its row
// (A) or column (B).
struct Split4 {
    bf16x4 h, m, l;
};
__device__ inline Split4 split4(double v0, double v1, double v2, double v3) {
    uint16_t h[4], m[4], l[4];
    split3(v0, h[0], m[0], l[0]);
    split3(v1, h[1], m[1], l[1]);
    split3(v2, h[2], m[2], l[2]);
    split3(v3, h[3], m[3], l[3]);
    Split4 s;
    s.h = bf16x4{(short)h[0], (short)h[1], (short)h[2], (short)h[3]};
    s.m = bf16x4{(short)m[0], (short)m[1], (short)m[2], (short)m[3]};
    s.l = bf16x4{(short)l[0], (short)l[1], (short)l[2], (short)l[3]};
    return s;
}

// acc += A B over one K step of 16 with the six-term product.  Lane layout
// (16x16x16): A[i][k] in lane 16 (k / 4) + i, element k % 4; B[k][j] in lane
// 16 (k / 4) + j, element k % 4; D[4 g + v][j] in element v of lane 16 g + j.
__device__ inline f32x4 mfma_bf16x6(const Split4& a, const Split4& b, f32x4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.m, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.m, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.l, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.l, b.h, acc, 0, 0, 0);
    return acc;
}

}  // namespace tt
