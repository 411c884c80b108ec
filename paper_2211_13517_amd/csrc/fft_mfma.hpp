// 1024-point inverse DFT of one wavefront in FP16 on the matrix cores: the
// inverse FFT of the frequency-domain correlation (section 2.2) with its
// dense stages in 16-bit arithmetic, as that section converts the
// convolution stage to a 16-bit format.
//
// The unnormalised inverse DFT y[k] = sum_n x[n] w^{nk}, w = exp(+2 pi i/1024),
// is split as n = 64 c + l, l = 16 t + 4 q + j, k = n' + 16 ka + 256 kb:
//   1. X1[k1][l] = sum_c x[64 c + l] w16^{c k1}  (64 DFTs of 16 points)
//   2. X1[k1][l] *= w^{l k1}
//   3. Y_j[ka][k1] = sum_{l'} X1[k1][4 l' + j] w16^{l' ka}, l' = 4 t + q
//      (64 DFTs of 16 points), then Y_j *= w64^{j ka}
//   4. y[k1 + 16 ka + 256 kb] = sum_j Y_j[ka][k1] w4^{j kb}  (radix 4, in lane)
// Stages 1 and 3 are dense 16 x 16 complex contractions, written as real
// products [re | im] x [[Re W, Im W], [-Im W, Re W]] with K = 32, each a
// v_mfma_f32_16x16x32_f16 (FP16 operands, FP32 sums).  The MFMA operand
// layout (A[i][k] in lane i + 16 (k/8), element k%8; B[k][j] in lane
// j + 16 (k/8), element k%8; D[i][j] in lane j + 16 (i/4), element i%4)
// makes the K index of both stages (q, element e) <-> (index q + 4 (e/2),
// part e%2), so one pair of weight registers serves as stage 1's B operand
// and stage 3's A operand.  Stage 1 takes its operand through a transpose
// across the four 16-lane rows in registers (v_permlane32_swap, then
// v_permlane16_swap); stage 3's operand is already where stage 1's results
// are.  Stage 1's results are rounded to FP16 pairs and twiddled in packed
// FP16 (v_pk_mul_f16, v_pk_fma_f16, FP16 table); the last twiddles and the
// radix-4 stage are FP32 vector arithmetic.
//
// Input: lane l (= 16 q + n) holds x[64 c + l] in h[c] (an FP16 pair).
// Output: y[e][kb] of lane (q, n) is y[n + 64 q + 16 e + 256 kb].
#pragma once
#include "common.hpp"

namespace fdas {
namespace mf {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTw2Stride = 20;  // FP16 pairs per lane of the stage-2 twiddle table (16 + 4 pad)
constexpr int kTw2Size = 64 * kTw2Stride;
constexpr int kTw3Size = 4 * 12;

// Two floats as an FP16 pair (round to nearest even), one v_cvt_pk_f16_f32.
__device__ __forceinline__ uint32_t pack_h2(float a, float b) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2));
}

// Per-lane DFT-16 weights: w0 (real outputs) and w1 (imaginary outputs) for
// lane (q, n), element e: index idx = q + 4 (e/2), part e%2, w = w16^{idx n}
// (FP64 phases, rounded to FP32 and then to FP16).
struct Weights {
  h8 w0, w1;
};

__device__ __forceinline__ Weights make_weights(int lane) {
  const int q = lane >> 4, n = lane & 15;
  Weights W;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int idx = q + 4 * (e >> 1);
    double s, c;
    sincospi(2.0 * (double)((idx * n) & 15) / 16.0, &s, &c);
    W.w0[e] = (_Float16)(float)((e & 1) ? -s : c);
    W.w1[e] = (_Float16)(float)((e & 1) ? c : s);
  }
  return W;
}

// Twiddle tables (FP64 phases rounded to FP32, and for tw2 then to FP16),
// filled by the block:
//   tw2[l * kTw2Stride + 4 j + t] = w^{n (16 t + 4 q + j)}  for lane l = 16 q + n (FP16 pairs)
//   tw3[12 q + 4 (j - 1) + e]     = w64^{j (4 q + e)}       for j = 1..3 (FP32)
__device__ __forceinline__ void fill_tables(uint32_t* tw2, c32* tw3, int tid, int nthreads) {
  for (int i = tid; i < 64 * 16; i += nthreads) {
    const int l = i >> 4, jt = i & 15, q = l >> 4, n = l & 15, j = jt >> 2, t = jt & 3;
    const int e = (n * (16 * t + 4 * q + j)) & 1023;
    double s, c;
    sincospi(2.0 * (double)e / 1024.0, &s, &c);
    tw2[l * kTw2Stride + jt] = pack_h2((float)c, (float)s);
  }
  for (int i = tid; i < kTw3Size; i += nthreads) {
    const int q = i / 12, j = (i % 12) / 4 + 1, e = i % 4;
    double s, c;
    sincospi(2.0 * (double)((j * (4 * q + e)) & 63) / 64.0, &s, &c);
    tw3[i] = {(float)c, (float)s};
  }
}

__device__ __forceinline__ c32 cmul_f(c32 a, c32 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// Complex product of FP16 pairs (real part in the low half) by two packed
// FP16 operations: (fr tr, fr ti), then + (-fi ti, fi tr).
__device__ __forceinline__ uint32_t cmul_h2(uint32_t f, uint32_t t) {
  const h2 a = __builtin_bit_cast(h2, f), b = __builtin_bit_cast(h2, t);
  const h2 p = h2{a.x, a.x} * b;
  const h2 r = __builtin_elementwise_fma(h2{-a.y, a.y}, h2{b.y, b.x}, p);
  return __builtin_bit_cast(uint32_t, r);
}

// x: the 16 input points of this lane as FP16 pairs (overwritten).
__device__ __forceinline__ void ifft1024(uint32_t (&h)[16], c32 (&y)[4][4], const uint32_t* tw2, const c32* tw3,
                                         const Weights& W, int lane) {
  const int q = lane >> 4, n = lane & 15;
  // stage 1 operands: chunk g of a lane is {x[c] : c = g, g + 4, g + 8, g + 12}
  // as FP16 pairs; lane (q, n) needs chunk q of lane (t, n) for t = 0..3, a
  // 4 x 4 transpose of (row, chunk) in each column n: rows 0-1 <-> 2-3 for
  // chunks (0, 2) and (1, 3), then rows 0 <-> 1 and 2 <-> 3 for chunks
  // (0, 1) and (2, 3), after which chunk t of lane (q, n) is chunk q of lane
  // (t, n)
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const auto r = __builtin_amdgcn_permlane32_swap(h[g + 4 * s], h[g + 2 + 4 * s], false, false);
      h[g + 4 * s] = r[0];
      h[g + 2 + 4 * s] = r[1];
    }
#pragma unroll
  for (int g = 0; g < 4; g += 2)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const auto r = __builtin_amdgcn_permlane16_swap(h[g + 4 * s], h[g + 1 + 4 * s], false, false);
      h[g + 4 * s] = r[0];
      h[g + 1 + 4 * s] = r[1];
    }
  f4 d0[4], d1[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    // instance l = 16 t + n of the stage-1 DFTs, elements c = q + 4 s
    const uint4 ch = {h[t], h[t + 4], h[t + 8], h[t + 12]};
    const h8 A = __builtin_bit_cast(h8, ch);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    d0[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, W.w0, z, 0, 0, 0);
    d1[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, W.w1, z, 0, 0, 0);
  }
  // d0[t][j] + i d1[t][j] = X1[k1 = n][l = 16 t + 4 q + j]; FP16 pairs,
  // twiddled in packed FP16, are stage 3's operand for each j (elements
  // t = 0..3)
  const uint4* twl = reinterpret_cast<const uint4*>(tw2 + lane * kTw2Stride);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint4 tj = twl[j];
    const uint32_t tt[4] = {tj.x, tj.y, tj.z, tj.w};
    uint32_t bb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) bb[t] = cmul_h2(pack_h2(d0[t][j], d1[t][j]), tt[t]);
    const uint4 b = {bb[0], bb[1], bb[2], bb[3]};
    const h8 B = __builtin_bit_cast(h8, b);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    const f4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.w0, B, z, 0, 0, 0);
    const f4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(W.w1, B, z, 0, 0, 0);
    // Y_j[ka = 4 q + e][k1 = n] = e0[e] + i e1[e]
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e][j] = {e0[e], e1[e]};
  }
  // twiddles w64^{j ka} and the radix-4 stage over j (w4 = +i)
  const c32* t3 = tw3 + 12 * q;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const c32 z0 = y[e][0], z1 = cmul_f(y[e][1], t3[e]), z2 = cmul_f(y[e][2], t3[4 + e]),
              z3 = cmul_f(y[e][3], t3[8 + e]);
    const c32 a = {z0.re + z2.re, z0.im + z2.im}, b = {z0.re - z2.re, z0.im - z2.im};
    const c32 c = {z1.re + z3.re, z1.im + z3.im}, d = {z1.re - z3.re, z1.im - z3.im};
    y[e][0] = {a.re + c.re, a.im + c.im};
    y[e][2] = {a.re - c.re, a.im - c.im};
    y[e][1] = {b.re - d.im, b.im + d.re};  // b + i d
    y[e][3] = {b.re + d.im, b.im - d.re};  // b - i d
  }
}

}  // namespace mf
}  // namespace fdas
