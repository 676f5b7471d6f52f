// Device-side constants and cross-file declarations of the HIP kernels' drivers.
#pragma once

#include "hf_internal.h"

namespace hf {

// 16x16x4 matrix-core products (wave64).  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register t of lane l holds C[row][l % 16] with
// row = 4 (l / 16) + t for f32 and row = l / 16 + 4 t for f64 (Mfma<T>::row).
typedef float hf_f4 __attribute__((ext_vector_type(4)));
typedef double hf_d4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<float> {
  using V = hf_f4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int t) { return 4 * (lane >> 4) + t; }
};
template <>
struct Mfma<double> {
  using V = hf_d4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int t) { return (lane >> 4) + 4 * t; }
};

// 64x64 output tile, 256 threads = 4 waves of 32x32 (2x2 blocks of 16x16):
// acc += As^T-staged A (64 x KC) times Bs-staged B (KC x 64), both stored k-major
// in LDS as [k][row] / [k][col].
template <class T, int KC, int LD>
__device__ __forceinline__ void mfma_tile_64(const T (*As)[LD], const T (*Bs)[LD],
                                             typename Mfma<T>::V acc[2][2], int lane, int wr, int wc) {
#pragma unroll
  for (int kk = 0; kk < KC; kk += 4) {
    const int k = kk + (lane >> 4);
    T a[2], b[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) a[bi] = As[k][wr + bi * 16 + (lane & 15)];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) b[bj] = Bs[k][wc + bj * 16 + (lane & 15)];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mfma<T>::mma(a[bi], b[bj], acc[bi][bj]);
  }
}

// FP16 operands for the matrix cores: 16x16x16 products with FP32 accumulation.
// Lane l supplies A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16], i < 4;
// the accumulator layout is the one of the FP32 16x16x4 product.
typedef _Float16 hf_h4 __attribute__((ext_vector_type(4)));

// Power of two s with max|x| * s < 2^14 (FP16's largest finite value is 65504):
// multiplying by s is exact, so the only rounding of a scaled operand is its cast.
__device__ __forceinline__ float fp16_scale(float mx) {
  if (!(mx > 0.f) || !(mx < 3.0e38f)) return 1.f;
  int e;
  (void)frexpf(mx, &e);  // mx = m 2^e, 0.5 <= m < 1
  return ldexpf(1.f, 14 - e);
}

// acc += (As scaled by sa)^T-staged A (64 x 16) times (Bs scaled by sb) (16 x 64)
// on the FP16 matrix cores, unscaled into the FP32 accumulator: one stage of 16
// values of k, staged in LDS as FP32 ([k][row] / [k][col]) like mfma_tile_64.
// SPLIT = false: every scaled operand is rounded to FP16 (11 significant bits).
// SPLIT = true: every scaled operand x is carried as the FP16 pair h + l,
// h = fp16(x), l = fp16(x - h) (about 22 significant bits), and the product as
// h_a h_b + h_a l_b + l_a h_b, three 16x16x16 products (the l_a l_b term is
// below the pair's own rounding).
template <int LD, bool SPLIT>
__device__ __forceinline__ void mfma_tile_64_h16(const float (*As)[LD], const float (*Bs)[LD], hf_f4 acc[2][2],
                                                 int lane, int wr, int wc, float sa, float sb) {
  const int k0 = 4 * (lane >> 4);
  hf_h4 a[2], b[2], al[2], bl[2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = As[k0 + i][wr + bi * 16 + (lane & 15)] * sa;
      a[bi][i] = (_Float16)x;
      if constexpr (SPLIT) al[bi][i] = (_Float16)(x - (float)a[bi][i]);
    }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float x = Bs[k0 + i][wc + bj * 16 + (lane & 15)] * sb;
      b[bj][i] = (_Float16)x;
      if constexpr (SPLIT) bl[bj][i] = (_Float16)(x - (float)b[bj][i]);
    }
  const float un = 1.f / (sa * sb);  // a power of two: exact
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      hf_f4 p = {0.f, 0.f, 0.f, 0.f};
      if constexpr (SPLIT) {
        p = __builtin_amdgcn_mfma_f32_16x16x16f16(a[bi], bl[bj], p, 0, 0, 0);
        p = __builtin_amdgcn_mfma_f32_16x16x16f16(al[bi], b[bj], p, 0, 0, 0);
      }
      p = __builtin_amdgcn_mfma_f32_16x16x16f16(a[bi], b[bj], p, 0, 0, 0);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[bi][bj][t] += p[t] * un;
    }
}

// Largest |value| of a staged 64 x 16 operand tile, from the four values each of
// the 256 threads staged: wave maxima through shuffles, then the four waves'
// maxima through `slot` (4 floats in LDS, read after the next barrier).
__device__ __forceinline__ void stage_max_post(float v, float* slot, int lane, int wave) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if (lane == 0) slot[wave] = v;
}
__device__ __forceinline__ float stage_max_read(const float* slot) {
  return fmaxf(fmaxf(slot[0], slot[1]), fmaxf(slot[2], slot[3]));
}

// Pipelined 64 x 64 tile product over k in [kbeg, kend), 256 threads:
// acc += A(0:64, k) B(k, 0:64).  Operands are fetched in stages of KB values of
// k into registers, so that the loads of stage s+1 are in flight while the
// matrix cores work on stage s (staged in LDS, As[k][row] / Bs[k][col]).
// fa(k, row) and fb(k, col) return the operand values (0 outside the tile);
// AKC selects the thread mapping of A's fetch: true when A is contiguous in k
// (consecutive threads take consecutive k), false when contiguous in row.
template <class T, int KB, int LD, bool AKC, class FA, class FB>
__device__ __forceinline__ void tile_gemm_64(typename Mfma<T>::V acc[2][2], T (*As)[LD], T (*Bs)[LD], int kbeg,
                                             int kend, FA&& fa, FB&& fb, int tid, int lane, int wr, int wc) {
  constexpr int NE = KB * 64 / 256;
  T ra[NE], rb[NE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + 256 * q;
      const int kq = AKC ? (e % KB) : (e >> 6);
      const int row = AKC ? (e / KB) : (e & 63);
      ra[q] = (k0 + kq < kend) ? fa(k0 + kq, row) : (T)0;
      const int kb = e >> 6, col = e & 63;
      rb[q] = (k0 + kb < kend) ? fb(k0 + kb, col) : (T)0;
    }
  };
  if (kbeg >= kend) return;
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + 256 * q;
      const int kq = AKC ? (e % KB) : (e >> 6);
      const int row = AKC ? (e / KB) : (e & 63);
      As[kq][row] = ra[q];
      Bs[e >> 6][e & 63] = rb[q];
    }
    __syncthreads();
    if (k0 + KB < kend) fetch(k0 + KB);
    mfma_tile_64<T, KB, LD>(As, Bs, acc, lane, wr, wc);
    __syncthreads();
  }
}

// stage of the pipelined sweeps' tile products (values of k per stage)
template <class T>
struct SweepStage {
  static constexpr int value = sizeof(T) == 4 ? 128 : 64;
};

template <class T>
void step1(hf_ctx* ctx, const double* values, hipStream_t s);


// inverses of the sweep step blocks of the L11 of every node of level l (the
// 64x64 diagonal inverses of the level formed first); they drive the TRSM of
// the level and the triangular sweeps
template <class T>
void step_inverses(hf_ctx* ctx, int l, hipStream_t s);

// explicit inverses of the whole L11 of every node of more than one sweep step
// (after step 1; recursive doubling of the step inverses)
template <class T>
void node_inverses(hf_ctx* ctx, hipStream_t s);

// Q^{-1} of Sec. 3.2: Y = (L D L^T)^{-1} R on the moderate part, R and Y row-major
// n x m in elimination order, FP64; factors in T.
template <class T>
// [lo, hi): rows outside hold no data of R (whole trees of a forest that the
// right-hand sides do not touch; their fronts are taken as zero, their rows of Y
// come out zero); hi < 0: all rows
void precond_apply(hf_ctx* ctx, int m, const double* R, double* Y, hipStream_t s, int64_t lo = 0, int64_t hi = -1);

}  // namespace hf
