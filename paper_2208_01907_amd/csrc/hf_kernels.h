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

template <class T>
void step1(hf_ctx* ctx, const double* values, hipStream_t s);


// inverses of the 64x64 diagonal blocks of L11, needed by precond_apply
template <class T>
void prepare_solve(hf_ctx* ctx, hipStream_t s);

// Q^{-1} of Sec. 3.2: Y = (L D L^T)^{-1} R on the moderate part, R and Y row-major
// n x m in elimination order, FP64; factors in T.
template <class T>
void precond_apply(hf_ctx* ctx, int m, const double* R, double* Y, hipStream_t s);

}  // namespace hf
