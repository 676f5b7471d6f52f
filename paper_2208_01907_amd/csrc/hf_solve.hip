// The preconditioner Q^{-1} of Sec. 3.2 on the GPU: forward and backward
// substitution with the low-precision factor of K11, multifrontal.
//
// Every tree node j owns an f_j x m block of a solve arena (T, row-major, m
// right-hand sides per row); its first rows are in pivot order.  Forward sweep,
// leaves first, per level:
//   gather   : own accepted rows from the FP64 input (cast to T), children's
//              border blocks added (extend-add, pivot-order aware);
//   steps of TB = 512 columns of L11:
//     diag   : z_J = L_JJ^{-1} w_J, a plain product with the inverse of the
//              512x512 step block, formed with each level of the
//              factorization (k_inv_diag for its 64x64 diagonal blocks,
//              k_inv_step for its two 256x256 halves, k_inv_merge for the block
//              below them; the TRSM of the level uses them too); z goes to a
//              second arena;
//     update : w_rows -= L[rows, J] z_J for every row below the step (the rest
//              of L11 and the border L21).
//   Launches over many fronts use 64-row tiles staged through LDS; launches
//   over few fronts use 16-row tiles fed straight from global memory.
//   A level with a node of more than one step runs in one pass instead: the
//   diagonal product with the explicit inverse of each node's whole L11 (formed
//   after step 1 from the step inverses), then one update of the border rows.
// Backward sweep, root first, per level:
//   border   : t = D^{-1} z - L21^T x_border (column strips, x_border read from
//              the FP64 result of the ancestors);
//   steps from the last one: diag (x_J = L_JJ^{-T} t_J with the same inverse,
//              scattered to FP64) and update of the columns left of the step
//              (one diagonal product with the node inverse on one-pass levels).
// Rows of the hard part are never written, so they stay zero in the result.
#include <algorithm>
#include <type_traits>

#include "hf_internal.h"
#include "hf_kernels.h"

namespace hf {

constexpr int TB = HF_SWEEP_STEP;  // columns of L11 per sweep step (512)
constexpr int HB = TB / 2;         // half step, inverted from the 64x64 inverses

// Inverse of the sweep step that starts at column J0 (a multiple of tb = TB or
// HB): the TB-block, or one of its diagonal halves; leading dimension TB.
template <class T>
__device__ __forceinline__ const T* step_inverse(const T* linv2, int64_t off, int J0) {
  const int h = (J0 % TB) / HB;
  return linv2 + off + (int64_t)(J0 / TB) * TB * TB + (int64_t)h * HB * TB + h * HB;
}

// Where a diagonal product of the sweeps finds its inverse: the step inverses,
// and (NODE: a level that runs in one pass) the explicit inverse of the whole
// L11 of every node of more than one step.  Without NODE the leading dimension
// is the constant TB.
template <class T>
struct InvSrc {
  const int64_t* off2;  // step inverses
  const T* linv2;
  const int64_t* noff;  // node inverses (offset < 0: the node has a single step)
  const int32_t* nld;
  const T* ninv;
};
// the inverse for the step at J0 of node j and its leading dimension (a node
// inverse is only asked for at J0 = 0)
template <bool NODE, class T>
__device__ __forceinline__ const T* inverse_of(const InvSrc<T>& v, int j, int J0, int& ld) {
  if constexpr (NODE) {
    const int64_t o = v.noff[j];
    if (o >= 0) {
      ld = v.nld[j];
      return v.ninv + o;
    }
  }
  ld = TB;
  return step_inverse(v.linv2, v.off2[j], J0);
}
constexpr int SB = 64;   // sub-block with an explicit inverse
constexpr int RCH = 512; // border rows per partial product of the backward sweep

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// leading dimension of the LDS stages of the sweeps' 64 x (<= 64) tile products
constexpr int MLD = 68;

template <class T>
__device__ __forceinline__ void zero_acc(typename Mfma<T>::V acc[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
}

// visit every (row, col, value) of a 64x64 accumulator tile
template <class T, class Fn>
__device__ __forceinline__ void for_tile(const typename Mfma<T>::V acc[2][2], int lane, int wr, int wc, Fn&& fn) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        fn(wr + bi * 16 + Mfma<T>::row(lane, t), wc + bj * 16 + (lane & 15), acc[bi][bj][t]);
}

// ---------------------------------------------------------------------------
// inverses of the 64x64 unit-lower diagonal blocks of every L11
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// inverse of every 256x256 step block, assembled from the 64x64 inverses:
// X_II = Linv_II, X_IJ = -Linv_II sum_{K=J}^{I-1} L_IK X_KJ  (I > J)
// ---------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(256)
k_inv_step(const int32_t* __restrict__ stp_node, const int32_t* __restrict__ stp_first,
           const NodeInfo* __restrict__ nodes, const NodeState* __restrict__ st,
           const T* __restrict__ front, const int64_t* __restrict__ linv_off, const T* __restrict__ linv,
           const int64_t* __restrict__ linv2_off, T* __restrict__ linv2, int base) {
  // one workgroup per (step, half, column block J): the block column J of the
  // half's inverse depends only on itself and L
  const int bi = base + (blockIdx.x >> 3), h = (blockIdx.x >> 2) & 1, J = blockIdx.x & 3;
  const int j = stp_node[bi];
  const int S = bi - stp_first[j];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int J0 = S * TB + h * HB;
  if (J0 >= npiv) return;
  const int nc = min(HB, npiv - J0);
  const int nb = (nc + SB - 1) / SB;
  if (J >= nb) return;
  const int64_t f = ni.f;
  const T* F = front + ni.front_off;
  T* X0 = linv2 + linv2_off[j] + (int64_t)S * TB * TB;  // column-major TB x TB step block
  T* X = X0 + (int64_t)h * HB * TB + h * HB;             // its diagonal half, leading dimension TB
  const T* L64 = linv + linv_off[j] + (int64_t)(J0 / SB) * SB * SB;
  __shared__ T As[32][64];
  __shared__ T Bs[32][64];
  __shared__ T Ts[64][64];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int e = tid; e < SB * TB; e += 256) X0[(int64_t)(h * HB + SB * J) * TB + e] = (T)0;  // the block's columns
  __syncthreads();
  for (int e = tid; e < SB * SB; e += 256) {
    const int r = e & 63, c = e >> 6;
    X[(int64_t)(SB * J + c) * TB + SB * J + r] = L64[(int64_t)J * SB * SB + (int64_t)c * SB + r];
  }
  __syncthreads();
  for (int I = J + 1; I < nb; ++I) {
    {
      T acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
      // stages of 32 values of k over K = J..I-1, each stage's operands fetched
      // into registers while the previous stage is multiplied
      const int nst = (I - J) * (SB / 32);
      T ra[8], rb[8];
      auto fetch = [&](int st2) {
        const int K = J + st2 / (SB / 32), k0 = (st2 % (SB / 32)) * 32;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid + 256 * q;
          const int r = e & 63, kq = e >> 6;
          const int gr = SB * I + r, gc = SB * K + k0 + kq;
          ra[q] = (gr < nc && gc < nc) ? F[(int64_t)(J0 + gc) * f + J0 + gr] : (T)0;
          const int kb = e & 31, c = e >> 5;
          rb[q] = X[(int64_t)(SB * J + c) * TB + SB * K + k0 + kb];
        }
      };
      fetch(0);
      for (int st2 = 0; st2 < nst; ++st2) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid + 256 * q;
          As[e >> 6][e & 63] = ra[q];
          Bs[e & 31][e >> 5] = rb[q];
        }
        __syncthreads();
        if (st2 + 1 < nst) fetch(st2 + 1);
#pragma unroll 4
        for (int kq = 0; kq < 32; ++kq) {
          T a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) { a[q] = As[kq][ty * 4 + q]; b[q] = Bs[kq][tx * 4 + q]; }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
        }
        __syncthreads();
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) Ts[ty * 4 + x][tx * 4 + y] = acc[x][y];
      __syncthreads();
      T out[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) out[a][b] = (T)0;
      const T* Li = L64 + (int64_t)I * SB * SB;
      for (int k0 = 0; k0 < SB; k0 += 32) {
        for (int e = tid; e < 32 * 64; e += 256) {
          const int r = e & 63, kq = e >> 6;
          As[kq][r] = Li[(int64_t)(k0 + kq) * SB + r];
        }
        __syncthreads();
#pragma unroll 4
        for (int kq = 0; kq < 32; ++kq) {
          T a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) { a[q] = As[kq][ty * 4 + q]; b[q] = Ts[k0 + kq][tx * 4 + q]; }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) out[x][y] += a[x] * b[y];
        }
        __syncthreads();
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          X[(int64_t)(SB * J + tx * 4 + y) * TB + SB * I + ty * 4 + x] = -out[x][y];
      __syncthreads();
    }
  }
}

// The block below the two halves of a step: X21 = -Linv_B L_BA Linv_A (A, B the
// halves).  Pass 0 forms P = L_BA Linv_A into the unused upper-right quarter
// (transposed: P(r, c) at quarter(c, r)); pass 1 forms X21 = -Linv_B P.  One
// workgroup per 64x64 output tile; all steps of one level in one launch.
template <class T>
__global__ void __launch_bounds__(256)
k_inv_merge(const int32_t* __restrict__ stp_node, const int32_t* __restrict__ stp_first,
            const NodeInfo* __restrict__ nodes, const NodeState* __restrict__ st,
            const T* __restrict__ front, const int64_t* __restrict__ linv2_off, T* __restrict__ linv2, int pass,
            int base) {
  const int bi = base + blockIdx.y;
  const int j = stp_node[bi];
  const int S = bi - stp_first[j];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int J0 = S * TB;
  const int nB = min(HB, npiv - J0 - HB);
  if (nB <= 0) return;
  const int rt = blockIdx.x >> 2, ct = blockIdx.x & 3;  // row tile (B), column tile (A)
  if (rt * 64 >= nB) return;
  const int64_t f = ni.f;
  const T* F = front + ni.front_off;
  T* X0 = linv2 + linv2_off[j] + (int64_t)S * TB * TB;
  constexpr int KB = SweepStage<T>::value / 2;
  __shared__ T As[KB][68];
  __shared__ T Bs[KB][68];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int r0 = rt * 64, c0 = ct * 64;
  const int nrow = min(64, nB - r0);
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = typename Mfma<T>::V{0, 0, 0, 0};
  // the zero triangles of Linv_A (k < c) and Linv_B (k > r) are skipped in whole
  // k stages (the stages keep their boundaries, so the sums are unchanged)
  if (pass == 0) {
    // P(r, c) = sum_{k >= c0} L[J0 + HB + r, J0 + k] Linv_A(k, c)
    tile_gemm_64<T, KB, 68, false>(
        acc, As, Bs, c0, HB,
        [&](int k, int r) { return r < nrow ? F[(int64_t)(J0 + k) * f + J0 + HB + r0 + r] : (T)0; },
        [&](int k, int c) { return X0[(int64_t)(c0 + c) * TB + k]; }, tid, lane, wr, wc);
  } else {
    // X21(r, c) = -sum_{k < r0 + 64} Linv_B(r, k) P(k, c), P(k, c) stored at X0[(HB + k) TB + c]
    tile_gemm_64<T, KB, 68, false>(
        acc, As, Bs, 0, min(nB, r0 + 64),
        [&](int k, int r) { return r < nrow ? X0[(int64_t)(HB + k) * TB + HB + r0 + r] : (T)0; },
        [&](int k, int c) { return X0[(int64_t)(HB + k) * TB + c0 + c]; }, tid, lane, wr, wc);
  }
#pragma unroll
  for (int bi2 = 0; bi2 < 2; ++bi2)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = wr + bi2 * 16 + Mfma<T>::row(lane, t), c = wc + bj * 16 + (lane & 15);
        if (r >= nrow) continue;
        if (pass == 0) X0[(int64_t)(HB + r0 + r) * TB + c0 + c] = acc[bi2][bj][t];
        else X0[(int64_t)(c0 + c) * TB + HB + r0 + r] = -acc[bi2][bj][t];
      }
}

// ---------------------------------------------------------------------------
// explicit inverse of the whole L11 of a node of more than one step, by
// recursive doubling: the diagonal blocks are the step inverses; blocks A, B of
// s columns each ([a0, a0 + s), [a0 + s, a0 + 2s)) merge as
// X_BA = -X_B L_BA X_A, for s = TB, 2 TB, ... until one block holds the node.
// Only the lower triangle is meaningful; P = L_BA X_A is kept, transposed, in
// the unused upper block (A rows, B columns) between the two passes.
// ---------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(256)
k_ninv_copy(const int32_t* __restrict__ steps, const int32_t* __restrict__ stp_node,
            const int32_t* __restrict__ stp_first, const NodeState* __restrict__ st,
            const int64_t* __restrict__ linv2_off, const T* __restrict__ linv2,
            const int64_t* __restrict__ ninv_off, const int32_t* __restrict__ ninv_ld, T* __restrict__ ninv,
            const int32_t* __restrict__ bad) {
  const int bi = steps[blockIdx.y];
  const int j = stp_node[bi];
  if (bad[j]) return;  // the sweeps keep the chains for this node
  const int S = bi - stp_first[j];
  const int J0 = S * TB;
  const int npiv = st[j].npiv;
  if (J0 >= npiv) return;
  const int nc = min(TB, npiv - J0);
  const int64_t ld = ninv_ld[j];
  const T* X = linv2 + linv2_off[j] + (int64_t)S * TB * TB;  // column-major TB x TB
  T* N = ninv + ninv_off[j] + (int64_t)J0 * ld + J0;
  // four consecutive rows of one column per thread
  const int e = 4 * (blockIdx.x * 256 + threadIdx.x);
  const int c = e / TB, r = e % TB;
  if (c >= nc || r >= nc) return;
  if (r + 3 < nc) {
    T v[4];
    __builtin_memcpy(v, X + (int64_t)c * TB + r, sizeof(v));
    __builtin_memcpy(N + (int64_t)c * ld + r, v, sizeof(v));
  } else {
    for (int q = r; q < nc; ++q) N[(int64_t)c * ld + q] = X[(int64_t)c * TB + q];
  }
}

// one 64 x 64 tile of P (pass 0) or of X_BA (pass 1) per workgroup; the
// products skip the zero triangles of X_A and X_B
template <class T>
__global__ void __launch_bounds__(256)
k_ninv_merge(const int32_t* __restrict__ jnode, const int32_t* __restrict__ ja0, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, const T* __restrict__ front, const int64_t* __restrict__ ninv_off,
             const int32_t* __restrict__ ninv_ld, T* __restrict__ ninv, const int32_t* __restrict__ bad, int sb,
             int pass, int base) {
  const int q = base + blockIdx.y;
  const int j = jnode[q], a0 = ja0[q], b0 = a0 + sb;
  if (bad[j]) return;
  const int npiv = st[j].npiv;
  const int nB = min(sb, npiv - b0);
  if (nB <= 0) return;
  const int nt = sb / 64;
  // pass 0 tiles P^T (rows: columns c of A), pass 1 tiles X_BA (rows: rows r of B)
  const int t0 = (blockIdx.x / nt) * 64, t1 = (blockIdx.x % nt) * 64;
  const int r0 = pass == 0 ? t1 : t0, c0 = pass == 0 ? t0 : t1;
  if (r0 >= nB) return;
  const int nrow = min(64, nB - r0);
  const NodeInfo ni = nodes[j];
  const int64_t f = ni.f, ld = ninv_ld[j];
  const T* F = front + ni.front_off;
  T* N = ninv + ninv_off[j];
  constexpr int KB = SweepStage<T>::value / 2;
  __shared__ T As[KB][68];
  __shared__ T Bs[KB][68];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  if (pass == 0) {
    // P^T(c, r) = sum_{k >= c0} X_A(k, c) L[b0 + r, a0 + k]: both operands are
    // fetched along their contiguous index (k for X_A, r for L)
    tile_gemm_64<T, KB, 68, true>(
        acc, As, Bs, c0, sb, [&](int k, int c) { return N[(int64_t)(a0 + c0 + c) * ld + a0 + k]; },
        [&](int k, int r) { return r < nrow ? F[(int64_t)(a0 + k) * f + b0 + r0 + r] : (T)0; }, tid, lane, wr, wc);
  } else {
    // X_BA(r, c) = -sum_{k < r0 + 64} X_B(r, k) P(k, c), P(k, c) at N[(b0 + k) ld + a0 + c]
    tile_gemm_64<T, KB, 68, false>(
        acc, As, Bs, 0, min(nB, r0 + 64),
        [&](int k, int r) { return r < nrow ? N[(int64_t)(b0 + k) * ld + b0 + r0 + r] : (T)0; },
        [&](int k, int c) { return N[(int64_t)(b0 + k) * ld + a0 + c0 + c]; }, tid, lane, wr, wc);
  }
  for_tile<T>(acc, lane, wr, wc, [&](int i, int jj, T v) {
    if (pass == 0) {
      if (jj < nrow) N[(int64_t)(b0 + r0 + jj) * ld + a0 + c0 + i] = v;  // P(r0 + jj, c0 + i)
    } else {
      if (i < nrow) N[(int64_t)(a0 + c0 + jj) * ld + b0 + r0 + i] = -v;  // X_BA(r0 + i, c0 + jj)
    }
  });
}

// Generation-stamped marks of one preconditioner application: live[j] = gen
// when front j gathered a nonzero forward block, tree[root] = gen when any front
// of that tree did.  A tree with no mark (a system of a block-diagonal forest
// that the right-hand sides do not touch) has z = 0 everywhere, hence x = 0: the
// backward sweep skips it (rootof null: a single tree, never skipped).
struct SweepMarks {
  int32_t* live;
  int32_t* tree;
  const int32_t* rootof;
  int gen;
  __device__ bool zero_tree(int j) const { return rootof && tree[rootof[j]] != gen; }
};

// ---------------------------------------------------------------------------
// forward sweep
// ---------------------------------------------------------------------------

// The forward gather of a level in one launch: every front row takes its own
// accepted value from the FP64 input (0 for postponed and border rows) plus the
// border rows of the children that map onto it, in child-rank order.  One
// thread per (assembly position, block of 16 right-hand sides), so the row's
// index loads serve its 16 values; own rows land at their pivot position.
template <class T>
__global__ void __launch_bounds__(256)
k_fwd_gather(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, const int32_t* __restrict__ ipos,
             const int64_t* __restrict__ gat_ptr, const int64_t* __restrict__ gat_src, int m,
             const double* __restrict__ R, T* __restrict__ rb, SweepMarks mk, int64_t rlo, int64_t rhi) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (ni.start >= rhi || ni.start + ni.p <= rlo) return;  // outside the rows that hold data: a zero front
  const int nch = (m + 15) >> 4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ni.f * nch) return;
  const int a = (int)(e / nch), c0 = 16 * (int)(e - (int64_t)a * nch);
  const int nc = min(16, m - c0);
  const int pr = a < ni.p ? ipos[ni.start + a] : a;
  T v[16];
  const bool own = a < ni.p && pr < npiv;
  const double* src0 = R + (int64_t)(ni.start + a) * m + c0;
  if (nc == 16) {  // whole blocks move in 16-byte pieces
#pragma unroll
    for (int c = 0; c < 16; c += 2) {
      double x[2] = {0.0, 0.0};
      if (own) __builtin_memcpy(x, src0 + c, 16);
      v[c] = (T)x[0];
      v[c + 1] = (T)x[1];
    }
  } else {
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = (own && c < nc) ? (T)src0[c] : (T)0;
  }
  const int64_t slot = ni.rhs_off + a;
  for (int64_t i = gat_ptr[slot]; i < gat_ptr[slot + 1]; ++i) {
    const T* src = rb + gat_src[i] * m + c0;
    if (nc == 16) {
      T x[16];
      __builtin_memcpy(x, src, 16 * sizeof(T));
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] += x[c];
    } else {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < nc) v[c] += src[c];
    }
  }
  // a front whose gathered block is all zero skips its forward products (a
  // right-hand side with few nonzero rows, such as the columns of K12)
  bool nz = false;
#pragma unroll
  for (int c = 0; c < 16; ++c) nz |= v[c] != (T)0;
  const unsigned long long anyw = __ballot(nz);  // one store per wave
  if (anyw && (int)(threadIdx.x & 63) == __ffsll((long long)anyw) - 1) {
    mk.live[j] = mk.gen;
    if (mk.rootof) mk.tree[mk.rootof[j]] = mk.gen;
  }
  T* dst = rb + (ni.rhs_off + pr) * m + c0;
  if (nc == 16) {
    __builtin_memcpy(dst, v, 16 * sizeof(T));
  } else {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < nc) dst[c] = v[c];
  }
}

// z_J = Linv_J w_J; four workgroups (64 rows each) per front, matrix cores
template <class T, int KB, bool NODE>
__global__ void __launch_bounds__(256)
k_fwd_diag(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
           const NodeState* __restrict__ st, InvSrc<T> inv, int J0, int tb, int m, const T* __restrict__ rb,
           T* __restrict__ zb, const int32_t* __restrict__ live, int gen) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv) return;
  const int nc = min(tb, npiv - J0);
  const int I = blockIdx.x;
  if (SB * I >= nc) return;
  if (live[j] != gen) {  // zero right-hand side block: z = 0
    T* Z0 = zb + (ni.rhs_off + J0 + SB * I) * m;
    for (int e = threadIdx.x; e < min(SB, nc - SB * I) * m; e += blockDim.x) Z0[e] = (T)0;
    return;
  }
  int ld;
  const T* X = inverse_of<NODE>(inv, j, J0, ld) + SB * I;
  const T* W = rb + (ni.rhs_off + J0) * m;
  __shared__ T As[KB][MLD];
  __shared__ T Bs[KB][MLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int nrows = min(SB, nc - SB * I);
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  const int cend = min(nc, SB * I + SB);
  tile_gemm_64<T, KB, MLD, false>(
      acc, As, Bs, 0, cend, [&](int k, int r) { return r < nrows ? X[(int64_t)k * ld + r] : (T)0; },
      [&](int k, int c) { return c < m ? W[(int64_t)k * m + c] : (T)0; }, tid, lane, wr, wc);
  T* Z = zb + (ni.rhs_off + J0 + SB * I) * m;
  for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
    if (r < nrows && c < m) Z[(int64_t)r * m + c] = v;
  });
}

// w_rows -= L[rows, J0:J0+nc] z_J for the rows below the step, 64-row strips
// (ONE: all pivots in one pass; the strips start at the border)
template <class T, int KB, bool ONE>
__global__ void __launch_bounds__(256)
k_fwd_upd(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
          const NodeState* __restrict__ st, const T* __restrict__ front, int J0, int tb, int m,
          const T* __restrict__ zb, T* __restrict__ rb, const int32_t* __restrict__ live, int gen) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv || live[j] != gen) return;
  const int nc = min(tb, npiv - J0);
  const int f = ni.f, p = ni.p;
  const int rs = (ONE ? p : J0 + nc) + blockIdx.x * 64;
  if (rs >= f) return;
  const int64_t lf = f;
  const T* A = front + ni.front_off + (int64_t)J0 * lf + rs;
  const T* Z = zb + (ni.rhs_off + J0) * m;
  T* W = rb + (ni.rhs_off + rs) * m;
  __shared__ T As[KB][MLD];
  __shared__ T Bs[KB][MLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int nrows = min(64, f - rs);
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  tile_gemm_64<T, KB, MLD, false>(
      acc, As, Bs, 0, nc, [&](int k, int r) { return r < nrows ? A[(int64_t)k * lf + r] : (T)0; },
      [&](int k, int c) { return c < m ? Z[(int64_t)k * m + c] : (T)0; }, tid, lane, wr, wc);
  for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
    const int gr = rs + r;
    if (r < nrows && c < m && !(gr >= npiv && gr < p)) W[(int64_t)r * m + c] -= v;
  });
}

// ---------------------------------------------------------------------------
// backward sweep
// ---------------------------------------------------------------------------

// Partial products P_ch[k] = sum_{r in chunk ch} L21[r, k] x_border[r] over
// chunks of RCH border rows (64-column strips x chunks x fronts); summed in a
// fixed order by k_bwd_border_fin.
// Border values of the backward sweep, gathered once per front from the FP64
// result into the front's (free) border rows of the sweep slab, in T.
template <class T>
__global__ void __launch_bounds__(256)
k_bwd_gather(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const int32_t* __restrict__ border, int m, const double* __restrict__ Y, T* __restrict__ rb,
             SweepMarks mk) {
  // one thread per (border row, block of 16 right-hand sides)
  const int j = lnodes[blockIdx.y];
  if (mk.zero_tree(j)) return;
  const NodeInfo ni = nodes[j];
  const int nch = (m + 15) >> 4;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ni.b * nch) return;
  const int r = (int)(e / nch), c0 = 16 * (int)(e - (int64_t)r * nch);
  const int nc = min(16, m - c0);
  const double* src = Y + (int64_t)border[ni.border_off + r] * m + c0;
  T* dst = rb + (ni.rhs_off + ni.p + r) * m + c0;
  if (nc == 16) {
    T v[16];
#pragma unroll
    for (int c = 0; c < 16; c += 2) {
      double x[2];
      __builtin_memcpy(x, src + c, 16);
      v[c] = (T)x[0];
      v[c + 1] = (T)x[1];
    }
    __builtin_memcpy(dst, v, 16 * sizeof(T));
  } else {
    for (int c = 0; c < nc; ++c) dst[c] = (T)src[c];
  }
}

// With FIN (every front of the level has one chunk) the product goes straight
// into t_k = z_k / d_k - P[k] (rows of the pivot block; the product reads the
// border rows).
template <class T, int KB, bool FIN>
__global__ void __launch_bounds__(256)
k_bwd_border_part(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
                  const NodeState* __restrict__ st, const T* __restrict__ front,
                  T* rb, int m, int maxch, int maxp, T* __restrict__ part, const T* __restrict__ dval,
                  const T* __restrict__ zb, SweepMarks mk) {
  const int q = blockIdx.z;
  const int j = lnodes[q];
  if (mk.zero_tree(j)) return;
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int cs = blockIdx.x * 64;
  const int ch = blockIdx.y;
  const int p = ni.p, b = ni.b;
  const int rlo = ch * RCH;
  if (cs >= npiv || rlo >= b) return;
  const int rhi = min(b, rlo + RCH);
  const int64_t lf = ni.f;
  const T* A = front + ni.front_off + (int64_t)cs * lf + p;  // A(k, r) = L21[r, cs + k]
  const T* Yb = rb + (ni.rhs_off + p) * m;  // border values, gathered by k_bwd_gather
  __shared__ T As[KB][MLD];
  __shared__ T Bs[KB][MLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int nrows = min(64, npiv - cs);
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  tile_gemm_64<T, KB, MLD, true>(
      acc, As, Bs, rlo, rhi, [&](int k, int r) { return r < nrows ? A[(int64_t)r * lf + k] : (T)0; },
      [&](int k, int c) { return c < m ? Yb[(int64_t)k * m + c] : (T)0; }, tid, lane, wr, wc);
  if constexpr (FIN) {
    for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
      if (r < nrows && c < m) {
        const int64_t o = (ni.rhs_off + cs + r) * m + c;
        rb[o] = zb[o] / dval[ni.start + cs + r] - v;
      }
    });
  } else {
    T* P = part + (((int64_t)q * maxch + ch) * maxp + cs) * m;
    for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
      if (r < nrows && c < m) P[(int64_t)r * m + c] = v;
    });
  }
}

// t_k = z_k / d_k - sum_ch P_ch[k]
template <class T>
__global__ void __launch_bounds__(256)
k_bwd_border_fin(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
                 const NodeState* __restrict__ st, const T* __restrict__ dval, int m, int maxch, int maxp,
                 const T* __restrict__ part, const T* __restrict__ zb, T* __restrict__ rb, SweepMarks mk) {
  const int q = blockIdx.y;
  const int j = lnodes[q];
  if (mk.zero_tree(j)) return;
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = (int)(e / m), col = (int)(e - (int64_t)k * m);
  if (k >= npiv) return;
  const int nch = (ni.b + RCH - 1) / RCH;
  T acc = (T)0;
  for (int ch = 0; ch < nch; ++ch) acc += part[(((int64_t)q * maxch + ch) * maxp + k) * m + col];
  const int64_t o = (ni.rhs_off + k) * m + col;
  rb[o] = zb[o] / dval[ni.start + k] - acc;
}

// x_J = Linv_J^T t_J (four workgroups of 64 columns), scattered to the FP64 result
template <class T, int KB, bool NODE>
__global__ void __launch_bounds__(256)
k_bwd_diag(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
           const NodeState* __restrict__ st, InvSrc<T> inv, const int32_t* __restrict__ piv, int J0, int tb,
           int m, double* __restrict__ Y, const T* __restrict__ rb, T* __restrict__ zb, SweepMarks mk) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv) return;
  const int nc = min(tb, npiv - J0);
  const int I = blockIdx.x;
  if (SB * I >= nc) return;
  if (mk.zero_tree(j)) {  // x = 0
    const int nr = min(SB, nc - SB * I), cz = J0 + SB * I;
    for (int e = threadIdx.x; e < nr * m; e += blockDim.x) {
      const int r = e / m, c = e - r * m;
      zb[(ni.rhs_off + cz + r) * m + c] = (T)0;
      Y[(int64_t)piv[ni.start + cz + r] * m + c] = 0.0;
    }
    return;
  }
  int ld;
  const T* X = inverse_of<NODE>(inv, j, J0, ld) + (int64_t)SB * I * ld;  // A(c, r) = X[c*ld + r]
  const T* W = rb + (ni.rhs_off + J0) * m;
  __shared__ T As[KB][MLD];
  __shared__ T Bs[KB][MLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int nrows = min(SB, nc - SB * I);
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  tile_gemm_64<T, KB, MLD, true>(
      acc, As, Bs, SB * I, nc, [&](int k, int r) { return r < nrows ? X[(int64_t)r * ld + k] : (T)0; },
      [&](int k, int c) { return c < m ? W[(int64_t)k * m + c] : (T)0; }, tid, lane, wr, wc);
  const int c0 = J0 + SB * I;
  for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
    if (r < nrows && c < m) {
      zb[(ni.rhs_off + c0 + r) * m + c] = v;
      Y[(int64_t)piv[ni.start + c0 + r] * m + c] = (double)v;
    }
  });
}

// t_k -= sum_{r in step} L[r, k] x_r for the columns k < J0 (64-column strips)
template <class T, int KB>
__global__ void __launch_bounds__(256)
k_bwd_upd(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
          const NodeState* __restrict__ st, const T* __restrict__ front, int J0, int tb, int m,
          const T* __restrict__ zb, T* __restrict__ rb, SweepMarks mk) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv || mk.zero_tree(j)) return;
  const int cs = blockIdx.x * 64;
  if (cs >= J0) return;
  const int nc = min(tb, npiv - J0);
  const int64_t lf = ni.f;
  const T* A = front + ni.front_off + (int64_t)cs * lf + J0;  // A(k, r) = L[J0 + r, cs + k]
  const T* Z = zb + (ni.rhs_off + J0) * m;
  T* W = rb + (ni.rhs_off + cs) * m;
  __shared__ T As[KB][MLD];
  __shared__ T Bs[KB][MLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int nrows = min(64, J0 - cs);
  typename Mfma<T>::V acc[2][2];
  zero_acc<T>(acc);
  tile_gemm_64<T, KB, MLD, true>(
      acc, As, Bs, 0, nc, [&](int k, int r) { return r < nrows ? A[(int64_t)r * lf + k] : (T)0; },
      [&](int k, int c) { return c < m ? Z[(int64_t)k * m + c] : (T)0; }, tid, lane, wr, wc);
  for_tile<T>(acc, lane, wr, wc, [&](int r, int c, T v) {
    if (r < nrows && c < m) W[(int64_t)r * m + c] -= v;
  });
}

// ---------------------------------------------------------------------------
// narrow launches: 16-row tiles fed straight from global memory
// ---------------------------------------------------------------------------
// Over few fronts a launch has few 64-row tiles, and a workgroup that streams a
// whole 64 x 512 block of L through its own CU is bound by the loads one CU
// keeps in flight.  These kernels cut the rows into 16-row tiles (four times
// the workgroups) and let the four waves of a workgroup take every fourth
// round of 16 values of k: a wave issues the loads of all its rounds (operands
// go straight into the matrix-core lane layout, no LDS staging) before its
// first product, and the four partial tiles are summed through LDS in wave
// order, so the result does not depend on timing.
//
// Rounds per wave: enough for a 512-value k range (8 rounds of 16 per wave).
template <class T>
struct NarrowRounds {  // rounds per batch, batches (register budget of FP64)
  static constexpr int NR = sizeof(T) == 4 ? 8 : 4;
  static constexpr int NBATCH = sizeof(T) == 4 ? 1 : 2;
};

// A(k .. k + 3, r) for an operand contiguous in k (col = the start of row r's
// values): one 4-element load where all four are below ke, else element by
// element with zeros from ke on
template <class T>
__device__ __forceinline__ typename Mfma<T>::V load4k(const T* __restrict__ col, int k, int ke) {
  typename Mfma<T>::V v = {0, 0, 0, 0};
  if (k + 3 < ke) {
    __builtin_memcpy(&v, col + k, 4 * sizeof(T));
    return v;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (k + s < ke) v[s] = col[k + s];
  return v;
}

// out(r, c) = sum_{kb <= k < ke} A(k, r) B(k, c) for r < 16, c < 16 NCB; the
// lane (i, g) = (lane % 16, lane / 16) of a wave supplies, in step s of round
// rd, the operands at k = kb + 16 rd + 4 g + s (the same k for A and B, so the
// k order inside a round is only a relabelling of the sum).  epi(r, c, v) is
// called once per output.  With CA (A contiguous in k), fa(k, r) returns the
// four values A(k .. k + 3, r), zero from ke on, in one load.
template <class T, int NCB, bool CA = false, bool LONG = false, class FA, class FB, class EPI>
__device__ __forceinline__ void narrow_product(int kb, int ke, FA&& fa, FB&& fb, EPI&& epi) {
  using V = typename Mfma<T>::V;
  constexpr int NR = NarrowRounds<T>::NR, NBATCH = NarrowRounds<T>::NBATCH;
  constexpr int NW = LONG ? 8 : 4;            // waves (LONG: two per SIMD, one's loads under the other's products)
  constexpr int KCH = 16 * NW * NR * NBATCH;  // values of k per pass
  static_assert(KCH >= TB, "one pass covers a step");
  __shared__ T red[NW][NCB][4][64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, g = lane >> 4;
  V acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = V{0, 0, 0, 0};
  // a step takes one pass; with LONG (a whole node inverse) a k range takes
  // several, in order of k
  for (int kc = kb; kc < ke; kc += KCH) {
#pragma unroll
  for (int bt = 0; bt < NBATCH; ++bt) {
    T a[NR][4], b[NR][NCB][4];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int k0 = kc + 16 * (w + NW * (bt * NR + q)) + 4 * g;
      if constexpr (CA) {
        const V a4 = fa(k0, li);
#pragma unroll
        for (int s = 0; s < 4; ++s) a[q][s] = a4[s];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool ok = k0 + s < ke;
        if constexpr (!CA) a[q][s] = ok ? fa(k0 + s, li) : (T)0;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[q][cb][s] = ok ? fb(k0 + s, cb * 16 + li) : (T)0;
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      if (kc + 16 * (w + NW * (bt * NR + q)) >= ke) break;  // uniform in the wave
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = Mfma<T>::mma(a[q][s], b[q][cb][s], acc[cb]);
    }
  }
  if constexpr (!LONG) break;
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int t = 0; t < 4; ++t) red[w][cb][t][lane] = acc[cb][t];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < (NCB * 4 + NW - 1) / NW; ++i) {
    const int e = tid + 64 * NW * i;
    if (e >= 256 * NCB) break;
    const int ln = e & 63, t = (e >> 6) & 3, cb = e >> 8;
    T v = red[0][cb][t][ln];
#pragma unroll
    for (int u = 1; u < NW; ++u) v += red[u][cb][t][ln];
    epi(Mfma<T>::row(ln, t), cb * 16 + (ln & 15), v);
  }
}

// Row tile of a narrow launch whose A operand runs along the rows (16 rows =
// 64 bytes in FP32, half a 128-byte line).  Workgroups go to the eight XCDs
// round-robin by their linear index, and each XCD has its own L2; the tiles are
// renumbered so that the two halves of a line (tiles 2i, 2i + 1) go to
// workgroups 8 apart, i.e. to the same XCD, and the line is fetched once.
__device__ __forceinline__ int xcd_pair_tile(int b, int n) {
  const int g = b >> 4;
  if (16 * g + 16 > n) return b;  // the last, partial group keeps its order
  return 16 * g + 2 * (b & 7) + ((b >> 3) & 1);
}

// z_J = Linv_J w_J, 16 rows of the step per workgroup
template <class T, int NCB, bool LONG>
__global__ void __launch_bounds__(LONG ? 512 : 256)
k_fwd_diag_n(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, InvSrc<T> inv, int J0, int tb, int m, const T* __restrict__ rb,
             T* __restrict__ zb, const int32_t* __restrict__ live, int gen) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv) return;
  const int nc = min(tb, npiv - J0);
  const int r0 = 16 * xcd_pair_tile(blockIdx.x, gridDim.x);
  if (r0 >= nc) return;
  const int nrows = min(16, nc - r0);
  if (live[j] != gen) {  // zero right-hand side block: z = 0
    T* Z0 = zb + (ni.rhs_off + J0 + r0) * m;
    for (int e = threadIdx.x; e < nrows * m; e += blockDim.x) Z0[e] = (T)0;
    return;
  }
  int ld;
  const T* X = inverse_of<LONG>(inv, j, J0, ld) + r0;  // A(k, r) = X[k ld + r]
  const T* W = rb + (ni.rhs_off + J0) * m;
  T* Z = zb + (ni.rhs_off + J0 + r0) * m;
  narrow_product<T, NCB, false, LONG>(
      0, min(nc, r0 + 16), [&](int k, int r) { return r < nrows ? X[(int64_t)k * ld + r] : (T)0; },
      [&](int k, int c) { return c < m ? W[(int64_t)k * m + c] : (T)0; },
      [&](int r, int c, T v) {
        if (r < nrows && c < m) Z[(int64_t)r * m + c] = v;
      });
}

// w_rows -= L[rows, J0:J0+nc] z_J for 16 rows below the step per workgroup
template <class T, int NCB, bool LONG>
__global__ void __launch_bounds__(LONG ? 512 : 256)
k_fwd_upd_n(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
            const NodeState* __restrict__ st, const T* __restrict__ front, int J0, int tb, int m,
            const T* __restrict__ zb, T* __restrict__ rb, const int32_t* __restrict__ live, int gen) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv || live[j] != gen) return;
  const int nc = min(tb, npiv - J0);
  const int f = ni.f, p = ni.p;
  // LONG (all pivots in one pass): the postponed rows [npiv, p) are skipped
  const int rs = (LONG ? p : J0 + nc) + 16 * xcd_pair_tile(blockIdx.x, gridDim.x);
  if (rs >= f) return;
  const int nrows = min(16, f - rs);
  const int64_t lf = f;
  const T* A = front + ni.front_off + (int64_t)J0 * lf + rs;  // A(k, r) = A[k lf + r]
  const T* Z = zb + (ni.rhs_off + J0) * m;
  T* W = rb + (ni.rhs_off + rs) * m;
  narrow_product<T, NCB, false, LONG>(
      0, nc, [&](int k, int r) { return r < nrows ? A[(int64_t)k * lf + r] : (T)0; },
      [&](int k, int c) { return c < m ? Z[(int64_t)k * m + c] : (T)0; },
      [&](int r, int c, T v) {
        const int gr = rs + r;
        if (r < nrows && c < m && !(gr >= npiv && gr < p)) W[(int64_t)r * m + c] -= v;
      });
}

// x_J = Linv_J^T t_J, 16 columns of the step per workgroup, scattered to the FP64 result
template <class T, int NCB, bool LONG>
__global__ void __launch_bounds__(LONG ? 512 : 256)
k_bwd_diag_n(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, InvSrc<T> inv, const int32_t* __restrict__ piv, int J0, int tb,
             int m, double* __restrict__ Y, const T* __restrict__ rb, T* __restrict__ zb, SweepMarks mk) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv) return;
  const int nc = min(tb, npiv - J0);
  const int r0 = 16 * blockIdx.x;
  if (r0 >= nc) return;
  const int nrows = min(16, nc - r0);
  if (mk.zero_tree(j)) {  // x = 0
    const int cz = J0 + r0;
    for (int e = threadIdx.x; e < nrows * m; e += blockDim.x) {
      const int r = e / m, c = e - r * m;
      zb[(ni.rhs_off + cz + r) * m + c] = (T)0;
      Y[(int64_t)piv[ni.start + cz + r] * m + c] = 0.0;
    }
    return;
  }
  int ld;
  const T* X = inverse_of<LONG>(inv, j, J0, ld) + (int64_t)r0 * ld;  // A(k, r) = X[r ld + k]
  const T* W = rb + (ni.rhs_off + J0) * m;
  const int c0 = J0 + r0;
  narrow_product<T, NCB, true, LONG>(
      r0, nc,
      [&](int k, int r) { return r < nrows ? load4k(X + (int64_t)r * ld, k, nc) : typename Mfma<T>::V{0, 0, 0, 0}; },
      [&](int k, int c) { return c < m ? W[(int64_t)k * m + c] : (T)0; },
      [&](int r, int c, T v) {
        if (r < nrows && c < m) {
          zb[(ni.rhs_off + c0 + r) * m + c] = v;
          Y[(int64_t)piv[ni.start + c0 + r] * m + c] = (double)v;
        }
      });
}

// t_k -= sum_{r in step} L[r, k] x_r for 16 columns k < J0 per workgroup
template <class T, int NCB>
__global__ void __launch_bounds__(256)
k_bwd_upd_n(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
            const NodeState* __restrict__ st, const T* __restrict__ front, int J0, int tb, int m,
            const T* __restrict__ zb, T* __restrict__ rb, SweepMarks mk) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (J0 >= npiv || mk.zero_tree(j)) return;
  const int cs = 16 * blockIdx.x;
  if (cs >= J0) return;
  const int nc = min(tb, npiv - J0);
  const int nrows = min(16, J0 - cs);
  const int64_t lf = ni.f;
  const T* A = front + ni.front_off + (int64_t)cs * lf + J0;  // A(k, r) = L[J0 + k, cs + r]
  const T* Z = zb + (ni.rhs_off + J0) * m;
  T* W = rb + (ni.rhs_off + cs) * m;
  narrow_product<T, NCB, true>(
      0, nc,
      [&](int k, int r) { return r < nrows ? load4k(A + (int64_t)r * lf, k, nc) : typename Mfma<T>::V{0, 0, 0, 0}; },
      [&](int k, int c) { return c < m ? Z[(int64_t)k * m + c] : (T)0; },
      [&](int r, int c, T v) {
        if (r < nrows && c < m) W[(int64_t)r * m + c] -= v;
      });
}

// ---------------------------------------------------------------------------
// whole fronts in one workgroup (FP32, at most 64 right-hand sides)
// ---------------------------------------------------------------------------
// On the lowest levels of the tree a level has many fronts (by default at least
// one per CU) of at most one sweep step (p <= TB); a workgroup takes a whole front
// through its forward or its backward step, one launch per level, with the
// right-hand-side block of the pivot rows in LDS.  The step uses the TB x TB
// inverse of the front's L11 (the same inverse as the level-wide launches):
//   forward : z = Linv w (pivot rows), w_border -= L21 z;
//   backward: t = z / d - L21^T x_border, x = Linv^T t.
// Products run on the matrix cores in 16-row tiles of NCB 16-column blocks
// (m <= 16 NCB); each output is summed in a fixed order (one wave, or per-wave
// partial sums added in wave order).
constexpr int FRONT_NT = 512;           // threads of a whole-front workgroup
constexpr int FRONT_NW = FRONT_NT / 64;
constexpr int FRONT_LDS = 160 * 1024;   // LDS of a workgroup (bytes)

// LDS row of 16 NCB right-hand sides, padded by 4 floats so that the four lane
// groups of a matrix-core operand read (rows 4 apart) hit different banks
template <int NCB>
struct FrontRow {
  static constexpr int W = 16 * NCB, LD = W + 4;
};
// rows of the backward step's LDS block: NCB = 1 keeps x_border and t side by
// side (b + p rows), wider blocks put t over x_border (max(b, p) rows)
template <int NCB>
struct FrontBwdRows {
  static constexpr int value = NCB == 1 ? 1024 : NCB == 2 ? 1024 : 576;
};
static_assert(FrontBwdRows<4>::value * FrontRow<4>::LD * 4 <= FRONT_LDS, "backward block fits LDS");
static_assert(FrontBwdRows<2>::value * FrontRow<2>::LD * 4 <= FRONT_LDS, "backward block fits LDS");

// acc[q][cb] += sum_{kb <= k < ke} A(k, 16 q + i) B(k, 16 cb + j) over one wave.
// A round covers 16 values of k in four matrix-core steps: lane (i, g) =
// (lane % 16, lane / 16) supplies A and B at k = k0 + 4 g + s in step s, so
// that the four values of A a lane needs in a round are consecutive in k.
// la(kq, r) returns A(kq .. kq + 3, r) with zeros from ke on; fb(k, c) reads B
// from LDS.  Batches of NR rounds are double-buffered: the loads of the next
// batch are in flight while the current one is multiplied.  kb is a multiple
// of 4.
template <int NA, int NCB, int NR, class LA, class FB>
__device__ __forceinline__ void wave_product(int kb, int ke, LA&& la, FB&& fb, hf_f4 (&acc)[NA][NCB]) {
  const int lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  constexpr int STEP = 16 * NR;
  hf_f4 a0[NR][NA], a1[NR][NA];
  float b0[NR][NCB][4], b1[NR][NCB][4];
  auto load = [&](int k0, hf_f4 (&a)[NR][NA], float (&bb)[NR][NCB][4]) {
#pragma unroll
    for (int rd = 0; rd < NR; ++rd) {
      const int kq = k0 + 16 * rd + 4 * g;
#pragma unroll
      for (int q = 0; q < NA; ++q) a[rd][q] = la(kq, 16 * q + li);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int s = 0; s < 4; ++s) bb[rd][cb][s] = kq + s < ke ? fb(kq + s, 16 * cb + li) : 0.f;
    }
  };
  auto comp = [&](int k0, const hf_f4 (&a)[NR][NA], const float (&bb)[NR][NCB][4]) {
#pragma unroll
    for (int rd = 0; rd < NR; ++rd) {
      if (k0 + 16 * rd >= ke) break;  // uniform in the wave
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = Mfma<float>::mma(a[rd][q][s], bb[rd][cb][s], acc[q][cb]);
    }
  };
  if (kb >= ke) return;
  load(kb, a0, b0);
  for (int k0 = kb; k0 < ke; k0 += 2 * STEP) {
    const bool more = k0 + STEP < ke;
    if (more) load(k0 + STEP, a1, b1);
    comp(k0, a0, b0);
    if (k0 + 2 * STEP < ke) load(k0 + 2 * STEP, a0, b0);
    if (more) comp(k0 + STEP, a1, b1);
  }
}

template <int NA, int NCB>
__device__ __forceinline__ void zero_tiles(hf_f4 (&acc)[NA][NCB]) {
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = hf_f4{0.f, 0.f, 0.f, 0.f};
}

// base[i] for a base shared by the wave and an index below 2^30: the byte
// offset fits 32 bits, so the load takes the base from scalar registers and a
// 32-bit offset per lane
__device__ __forceinline__ float ld_off(const float* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (i << 2));
}

// A values for the lane's four consecutive k when A(k, r) = base[o + k] (o the
// lane's row offset; contiguous in k): one 16-byte load where all four are in
// range.  Offsets stay below 2^30 (small fronts).
__device__ __forceinline__ hf_f4 load4_contig(const float* __restrict__ base, uint32_t o, int kq, int ke,
                                              bool row_ok) {
  hf_f4 v = hf_f4{0.f, 0.f, 0.f, 0.f};
  if (!row_ok) return v;
  if (kq + 3 < ke) {
    __builtin_memcpy(&v, reinterpret_cast<const char*>(base) + ((o + (uint32_t)kq) << 2), 16);
    return v;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = kq + s < ke ? ld_off(base, o + (uint32_t)(kq + s)) : 0.f;
  return v;
}

// ... when A(k, r) = base[o + k ld] (rows contiguous across lanes)
__device__ __forceinline__ hf_f4 load4_strided(const float* __restrict__ base, uint32_t o, uint32_t ld, int kq,
                                                int ke, bool row_ok) {
  hf_f4 v;
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = (row_ok && kq + s < ke) ? ld_off(base, o + (uint32_t)(kq + s) * ld) : 0.f;
  return v;
}

typedef double hf_d2 __attribute__((ext_vector_type(2)));

// One row of m <= W right-hand sides, widened to W with zeros: FP64 input (cast
// to FP32; zeros when !on), FP32 accumulation and store.  Rows of m = W values
// are 16-byte aligned and move in 16-byte pieces.
template <int W>
__device__ __forceinline__ void load_row(const double* __restrict__ src, int64_t off, int m, bool on,
                                         float (&v)[W]) {
#pragma unroll
  for (int c = 0; c < W; ++c) v[c] = 0.f;
  if (!on) return;
  if (m == W) {
    const hf_d2* q = reinterpret_cast<const hf_d2*>(src + off);
#pragma unroll
    for (int c = 0; c < W / 2; ++c) {
      const hf_d2 x = q[c];
      v[2 * c] = (float)x[0];
      v[2 * c + 1] = (float)x[1];
    }
  } else {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c < m) v[c] = (float)src[off + c];
  }
}
template <int W>
__device__ __forceinline__ void add_row(const float* __restrict__ src, int m, float (&v)[W]) {
  if (m == W) {
    const hf_f4* q = reinterpret_cast<const hf_f4*>(src);
#pragma unroll
    for (int c = 0; c < W / 4; ++c) {
      const hf_f4 x = q[c];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[4 * c + u] += x[u];
    }
  } else {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c < m) v[c] += src[c];
  }
}
template <int W>
__device__ __forceinline__ void store_row(float* __restrict__ dst, int m, const float (&v)[W]) {
  if (m == W) {
    hf_f4* q = reinterpret_cast<hf_f4*>(dst);
#pragma unroll
    for (int c = 0; c < W / 4; ++c) q[c] = hf_f4{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
  } else {
#pragma unroll
    for (int c = 0; c < W; ++c)
      if (c < m) dst[c] = v[c];
  }
}

// tile visited by wave w in its round q when the tiles' costs grow (or shrink)
// with their index: alternate directions so every wave gets a similar sum
__device__ __forceinline__ int snake_tile(int w, int q) {
  return FRONT_NW * q + ((q & 1) ? FRONT_NW - 1 - w : w);
}

// Forward step of a whole front: gather (own accepted rows from the FP64 input,
// children's border rows added in child-rank order), z = Linv w for the pivot
// rows (to zb and LDS), then w_border -= L21 z.  One column block: z has its
// own LDS block and the border product runs in 64-row tiles whose k range is
// split over the waves, the eight partial sums added in wave order (in the LDS
// of w).  Wider blocks: z replaces w in LDS and each wave takes whole 16-row
// tiles of the border.  Postponed rows are not part of the moderate solve and
// are not written.
template <int NCB>
__global__ void __launch_bounds__(FRONT_NT)
k_fwd_front(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
            const NodeState* __restrict__ st, const int32_t* __restrict__ ipos,
            const int64_t* __restrict__ gat_ptr, const int64_t* __restrict__ gat_src, int m,
            const double* __restrict__ R, const float* __restrict__ front, const int64_t* __restrict__ linv2_off,
            const float* __restrict__ linv2, float* __restrict__ rb, float* __restrict__ zb, SweepMarks mk,
            int64_t rlo, int64_t rhi) {
  constexpr int MT = TB / 16 / FRONT_NW;  // 16-row tiles of the pivot block per wave
  constexpr int W = FrontRow<NCB>::W, LD = FrontRow<NCB>::LD;
  constexpr bool SPLIT = NCB == 1;
  __shared__ float ws[TB][LD];                 // w of the pivot rows (then z, or the partial sums)
  __shared__ float zsep[SPLIT ? TB : 1][LD];   // z of the pivot rows (one column block)
  static_assert(!SPLIT || FRONT_NW * 64 * 16 <= TB * LD, "partial sums fit in ws");
  float(*zs)[LD] = SPLIT ? zsep : ws;
  const int j = lnodes[blockIdx.x];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int f = ni.f, p = ni.p, b = ni.b;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15;
  if (ni.start >= rhi || ni.start + p <= rlo) {  // outside the rows that hold data: z = 0
    float* Z = zb + ni.rhs_off * m;
    for (int e = tid; e < npiv * m; e += FRONT_NT) Z[e] = 0.f;
    return;
  }
  // one thread per front row: every load of a row is issued at once
  int nz = 0;
  for (int a = tid; a < f; a += FRONT_NT) {
    const int pr = a < p ? ipos[ni.start + a] : a;
    if (pr >= npiv && pr < p) continue;
    float v[W];
    load_row<W>(R, (int64_t)(ni.start + a) * m, m, a < p, v);
    const int64_t slot = ni.rhs_off + a;
    for (int64_t i = gat_ptr[slot]; i < gat_ptr[slot + 1]; ++i) add_row<W>(rb + gat_src[i] * m, m, v);
#pragma unroll
    for (int c = 0; c < W; ++c) nz |= v[c] != 0.f;
    if (pr < npiv) {
#pragma unroll
      for (int c = 0; c < W; ++c) ws[pr][c] = v[c];
    } else {
      store_row<W>(rb + (ni.rhs_off + pr) * m, m, v);
    }
  }
  // an all-zero block (a right-hand side with few nonzero rows, such as the
  // columns of K12): z = 0, and the border rows keep the zeros just stored
  if (!__syncthreads_or(nz)) {
    float* Z = zb + ni.rhs_off * m;
    for (int e = tid; e < npiv * m; e += FRONT_NT) Z[e] = 0.f;
    return;
  }
  if (tid == 0 && mk.rootof) mk.tree[mk.rootof[j]] = mk.gen;
  const float* X = linv2 + linv2_off[j];  // the front's single step, column-major TB x TB
  const int ntile = (npiv + 15) / 16;
  hf_f4 zt[MT][1][NCB];
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    zero_tiles(zt[q]);
    const int t = snake_tile(w, q);
    if (t >= ntile) continue;
    const int r0 = 16 * t;
    const bool row_ok = r0 + li < npiv;
    const int ke = min(npiv, r0 + 16);
    wave_product<1, NCB, SPLIT ? 2 : 1>(
        0, ke, [&](int kq, int r) { return load4_strided(X, (uint32_t)(r0 + r), TB, kq, ke, row_ok); },
        [&](int k, int c) { return ws[k][c]; }, zt[q]);
  }
  if constexpr (!SPLIT) __syncthreads();  // every read of w is done: z replaces it
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const int t = snake_tile(w, q);
    if (t >= ntile) continue;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = 16 * t + Mfma<float>::row(lane, u), c = 16 * cb + li;
        if (r < npiv) {
          zs[r][c] = zt[q][0][cb][u];
          if (c < m) zb[(ni.rhs_off + r) * m + c] = zt[q][0][cb][u];
        }
      }
  }
  __syncthreads();
  const float* F = front + ni.front_off;
  if constexpr (SPLIT) {
    const int kc = ((npiv + FRONT_NW - 1) / FRONT_NW + 15) & ~15;  // k range of one wave
    const int kb = min(npiv, w * kc), ke = min(npiv, kb + kc);
    float* part = &ws[0][0];  // [wave][64 rows][16]
    for (int r0 = 0; r0 < b; r0 += 64) {
      hf_f4 acc[4][1];
      zero_tiles(acc);
      // A(k, r) = F[p + r0 + r + k f]
      wave_product<4, 1, 1>(
          kb, ke, [&](int kq, int r) { return load4_strided(F, (uint32_t)(p + r0 + r), f, kq, ke, r0 + r < b); },
          [&](int k, int c) { return zs[k][c]; }, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) part[(w * 64 + 16 * q + Mfma<float>::row(lane, u)) * 16 + li] = acc[q][0][u];
      __syncthreads();
      for (int e = tid; e < 64 * 16; e += FRONT_NT) {
        const int r = e >> 4, c = e & 15;
        if (r0 + r < b && c < m) {
          float sum = 0.f;
#pragma unroll
          for (int v = 0; v < FRONT_NW; ++v) sum += part[(v * 64 + r) * 16 + c];
          rb[(ni.rhs_off + p + r0 + r) * m + c] -= sum;
        }
      }
      __syncthreads();
    }
  } else {
    for (int r0 = 16 * w; r0 < b; r0 += 16 * FRONT_NW) {
      hf_f4 acc[1][NCB];
      zero_tiles(acc);
      const bool row_ok = r0 + li < b;
      wave_product<1, NCB, 1>(
          0, npiv, [&](int kq, int r) { return load4_strided(F, (uint32_t)(p + r0 + r), f, kq, npiv, row_ok); },
          [&](int k, int c) { return zs[k][c]; }, acc);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + Mfma<float>::row(lane, u), c = 16 * cb + li;
          if (r < b && c < m) rb[(ni.rhs_off + p + r) * m + c] -= acc[0][cb][u];
        }
    }
  }
}

// Backward step of a whole front: x_border gathered from the FP64 result of the
// ancestors into LDS, t = z / d - L21^T x_border for the pivot rows (LDS: after
// the border rows for one column block, over them for wider blocks), then
// x = Linv^T t scattered to the FP64 result.
template <int NCB>
__global__ void __launch_bounds__(FRONT_NT)
k_bwd_front(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
            const NodeState* __restrict__ st, const float* __restrict__ front,
            const int64_t* __restrict__ linv2_off, const float* __restrict__ linv2, const int32_t* __restrict__ piv,
            const int32_t* __restrict__ border, const float* __restrict__ dval, int m, double* __restrict__ Y,
            const float* __restrict__ zb, SweepMarks mk) {
  constexpr int MT = TB / 16 / FRONT_NW;
  constexpr int W = FrontRow<NCB>::W, LD = FrontRow<NCB>::LD;
  __shared__ float sh[FrontBwdRows<NCB>::value][LD];
  const int j = lnodes[blockIdx.x];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  if (mk.zero_tree(j)) {  // x = 0
    for (int e = threadIdx.x; e < npiv * m; e += FRONT_NT) {
      const int r = e / m, c = e - r * m;
      Y[(int64_t)piv[ni.start + r] * m + c] = 0.0;
    }
    return;
  }
  const int f = ni.f, p = ni.p, b = ni.b;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15;
  if (npiv == 0) return;
  for (int r = tid; r < b; r += FRONT_NT) {
    float v[W];
    load_row<W>(Y, (int64_t)border[ni.border_off + r] * m, m, true, v);
#pragma unroll
    for (int c = 0; c < W; ++c) sh[r][c] = v[c];
  }
  __syncthreads();
  const float* F = front + ni.front_off;
  const int ntile = (npiv + 15) / 16;
  hf_f4 tt[MT][1][NCB];
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    zero_tiles(tt[q]);
    const int t = w + FRONT_NW * q;
    if (t >= ntile) continue;
    const int r0 = 16 * t;
    const bool row_ok = r0 + li < npiv;
    const uint32_t o = (uint32_t)(r0 + li) * f + p;  // L21[k, r0 + li] = F[o + k]
    wave_product<1, NCB, NCB == 1 ? 4 : 2>(
        0, b, [&](int kq, int) { return load4_contig(F, o, kq, b, row_ok); },
        [&](int k, int c) { return sh[k][c]; }, tt[q]);
  }
  float(*ts)[LD] = NCB == 1 ? sh + b : sh;
  if constexpr (NCB > 1) __syncthreads();  // every read of x_border is done: t replaces it
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const int t = w + FRONT_NW * q;
    if (t >= ntile) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 16 * t + Mfma<float>::row(lane, u);
      if (r >= npiv) continue;
      const float dk = dval[ni.start + r];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int c = 16 * cb + li;
        ts[r][c] = c < m ? zb[(ni.rhs_off + r) * m + c] / dk - tt[q][0][cb][u] : 0.f;
      }
    }
  }
  __syncthreads();
  const float* X = linv2 + linv2_off[j];
#pragma unroll
  for (int q = 0; q < MT; ++q) {
    const int t = snake_tile(w, q);
    if (t >= ntile) continue;
    const int r0 = 16 * t;
    const bool row_ok = r0 + li < npiv;
    hf_f4 acc[1][NCB];
    zero_tiles(acc);
    const uint32_t o = (uint32_t)(r0 + li) * TB;  // Linv[k, r0 + li] = X[o + k]
    wave_product<1, NCB, NCB == 1 ? 4 : 2>(
        r0, npiv, [&](int kq, int) { return load4_contig(X, o, kq, npiv, row_ok); },
        [&](int k, int c) { return ts[k][c]; }, acc);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + Mfma<float>::row(lane, u), c = 16 * cb + li;
        if (r < npiv && c < m) Y[(int64_t)piv[ni.start + r] * m + c] = (double)acc[0][cb][u];
      }
  }
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------

template <class T>
void step_inverses(hf_ctx* ctx, int l, hipStream_t s) {
  const int base = ctx->lvl_step_ptr[l], ns = ctx->lvl_step_ptr[l + 1] - base;
  if (ns <= 0) return;
  launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_inv_step<T>, dim3((unsigned)(8 * ns)), dim3(256),
               (const int32_t*)ctx->d_stp_node.as<int32_t>(), (const int32_t*)ctx->d_stp_first.as<int32_t>(),
               (const NodeInfo*)ctx->d_nodes.as<NodeInfo>(), (const NodeState*)ctx->d_state.as<NodeState>(),
               (const T*)ctx->d_front.as<T>(), (const int64_t*)ctx->d_linv_off.as<int64_t>(),
               (const T*)ctx->d_linv.as<T>(), (const int64_t*)ctx->d_linv2_off.as<int64_t>(), ctx->d_linv2.as<T>(),
               base);
  for (int pass = 0; pass < 2; ++pass)
    launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_inv_merge<T>, dim3(16, (unsigned)ns), dim3(256),
                 (const int32_t*)ctx->d_stp_node.as<int32_t>(), (const int32_t*)ctx->d_stp_first.as<int32_t>(),
                 (const NodeInfo*)ctx->d_nodes.as<NodeInfo>(), (const NodeState*)ctx->d_state.as<NodeState>(),
                 (const T*)ctx->d_front.as<T>(), (const int64_t*)ctx->d_linv2_off.as<int64_t>(), ctx->d_linv2.as<T>(),
                 pass, base);
}

// Sign test of the L11 of a node of more than one step (one wave per column):
// bad[j] is set when a strictly lower entry of column c is positive.  An L11 with
// no positive entry below the diagonal (the factor of an M-matrix, such as a
// diffusion operator) has an inverse with no negative entry, so the products
// with the node inverse add terms of one sign; otherwise they can cancel, and
// the sweeps keep the chains of steps (substitution does not lose accuracy to
// that cancellation).  Order-independent: the flag is only ever raised.
template <class T>
__global__ void __launch_bounds__(256)
k_l11_sign(int ncols, const int32_t* __restrict__ cnode, const int32_t* __restrict__ ccol,
           const NodeInfo* __restrict__ nodes, const NodeState* __restrict__ st, const T* __restrict__ front,
           int32_t* __restrict__ bad) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= ncols) return;
  const int j = cnode[q], c = ccol[q];
  const int npiv = st[j].npiv;
  const NodeInfo ni = nodes[j];
  const T* L = front + ni.front_off + (int64_t)c * ni.f;
  bool pos = false;
  for (int r = c + 1 + lane; r < npiv; r += 64) pos |= L[r] > (T)0;
  if (__any(pos) && lane == 0) atomicOr(bad + j, 1);
}

template <class T>
void node_inverses(hf_ctx* ctx, hipStream_t s) {
  if (ctx->ninv_copy.empty()) return;
  const NodeState* st = ctx->d_state.as<NodeState>();
  T* ninv = ctx->d_ninv.as<T>();
  const int64_t* noff = ctx->d_ninv_off.as<int64_t>();
  const int32_t* nld = ctx->d_ninv_ld.as<int32_t>();
  // FP32, default mode: the sign test decides which nodes get an inverse
  int32_t* bad = ctx->d_ninv_bad.as<int32_t>();
  HF_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t) * ctx->n_nodes, s));
  if (ctx->opt.sweep_node_inverse == 1 && std::is_same<T, float>::value) {
    const int ncols = (int)ctx->ninv_cnode.size();
    launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_l11_sign<T>, dim3(cdiv(ncols, 4)), dim3(256), ncols,
                 (const int32_t*)ctx->d_ninv_cnode.as<int32_t>(), (const int32_t*)ctx->d_ninv_ccol.as<int32_t>(),
                 (const NodeInfo*)ctx->d_nodes.as<NodeInfo>(), st, (const T*)ctx->d_front.as<T>(), bad);
  }
  launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_ninv_copy<T>,
               dim3(TB * TB / 1024, (unsigned)ctx->ninv_copy.size()), dim3(256),
               (const int32_t*)ctx->d_ninv_copy.as<int32_t>(), (const int32_t*)ctx->d_stp_node.as<int32_t>(),
               (const int32_t*)ctx->d_stp_first.as<int32_t>(), st, (const int64_t*)ctx->d_linv2_off.as<int64_t>(),
               (const T*)ctx->d_linv2.as<T>(), noff, nld, ninv, (const int32_t*)bad);
  for (size_t t = 0; t + 1 < ctx->ninv_lvl.size(); ++t) {
    const int base = ctx->ninv_lvl[t], nj = ctx->ninv_lvl[t + 1] - base;
    if (nj <= 0) continue;
    const int sb = TB << t;
    for (int pass = 0; pass < 2; ++pass)
      launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_ninv_merge<T>,
                   dim3((unsigned)((sb / 64) * (sb / 64)), (unsigned)nj), dim3(256),
                   (const int32_t*)ctx->d_ninv_jnode.as<int32_t>(), (const int32_t*)ctx->d_ninv_ja0.as<int32_t>(),
                   (const NodeInfo*)ctx->d_nodes.as<NodeInfo>(), st, (const T*)ctx->d_front.as<T>(), noff, nld, ninv,
                   (const int32_t*)bad, sb, pass, base);
  }
}

// border product of the backward sweep for 16 pivot rows per workgroup (narrow
// form of k_bwd_border_part: operands loaded straight into MFMA registers)
template <class T, int NCB, bool FIN>
__global__ void __launch_bounds__(256)
k_bwd_border_n(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
               const NodeState* __restrict__ st, const T* __restrict__ front,
               T* rb, int m, int maxch, int maxp, T* __restrict__ part, const T* __restrict__ dval,
               const T* __restrict__ zb, SweepMarks mk) {
  const int q = blockIdx.z;
  const int j = lnodes[q];
  if (mk.zero_tree(j)) return;
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int cs = blockIdx.x * 16;
  const int ch = blockIdx.y;
  const int p = ni.p, b = ni.b;
  const int rlo = ch * RCH;
  if (cs >= npiv || rlo >= b) return;
  const int rhi = min(b, rlo + RCH);
  const int64_t lf = ni.f;
  const T* A = front + ni.front_off + (int64_t)cs * lf + p;  // A(k, r) = L21[k, cs + r]
  const T* Yb = rb + (ni.rhs_off + p) * m;
  const int nrows = min(16, npiv - cs);
  T* P = part + (((int64_t)q * maxch + ch) * maxp + cs) * m;
  narrow_product<T, NCB, true>(
      rlo, rhi,
      [&](int k, int r) { return r < nrows ? load4k(A + (int64_t)r * lf, k, rhi) : typename Mfma<T>::V{0, 0, 0, 0}; },
      [&](int k, int c) { return c < m ? Yb[(int64_t)k * m + c] : (T)0; },
      [&](int r, int c, T v) {
        if (r < nrows && c < m) {
          if constexpr (FIN) {
            const int64_t o = (ni.rhs_off + cs + r) * m + c;
            rb[o] = zb[o] / dval[ni.start + cs + r] - v;
          } else {
            P[(int64_t)r * m + c] = v;
          }
        }
      });
}

__global__ void k_zero_rows(int M, int m, const int32_t* __restrict__ rows, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * m) return;
  const int64_t i = e / m;
  Y[(int64_t)rows[i] * m + (e - i * m)] = 0.0;
}

template <class T>
void precond_apply(hf_ctx* ctx, int m, const double* R, double* Y, hipStream_t s, int64_t lo, int64_t hi) {
  const int64_t rlo = lo, rhi = hi < 0 ? ctx->n : hi;
  if (m < 1 || m > 64) throw Status{HF_ERR_ARG};  // the sweep tiles hold at most 64 columns
  // Stage sizes of the tile products: launches over few fronts are latency
  // bound (one workgroup per CU, long stages, few round trips); launches over
  // many fronts are throughput bound (short stages, several workgroups per CU).
  constexpr int KBN = SweepStage<T>::value;
  constexpr int KBW = SweepStage<T>::value / 4;
  const int64_t wide_min = ctx->opt.sweep_wide_min;
  auto wide = [&](const dim3& g) { return (int64_t)g.x * g.y * g.z >= wide_min; };
  // step length: long steps (fewer sequential launches) over few fronts,
  // half steps (shorter diagonal products) over many
  auto step_of = [](int nl) { return nl < 128 ? TB : HB; };
  // narrow launches run the 16-row kernels with the fewest column blocks that
  // hold m
  const int ncb = m <= 16 ? 1 : m <= 32 ? 2 : 4;
  auto pick = [&](auto k1, auto k2, auto k4) { return ncb == 1 ? k1 : ncb == 2 ? k2 : k4; };
  const int nlev = (int)ctx->level_ptr.size() - 1;
  const size_t arena = (size_t)std::max<int64_t>(ctx->rhs_rows, 1) * m * sizeof(T);
  ctx->d_rhs_arena.alloc(arena);
  ctx->d_zb_arena.alloc(arena);
  T* rb = ctx->d_rhs_arena.as<T>();
  T* zb = ctx->d_zb_arena.as<T>();
  const T* front = ctx->d_front.as<T>();
  const T* linv2 = ctx->d_linv2.as<T>();
  const int64_t* loff2 = ctx->d_linv2_off.as<int64_t>();
  // levels with a node of more than one step take each direction in one pass
  // over the node inverses where step 1 formed them for all such nodes of the
  // level (level_one_pass, set after step 1 from the sign test of L11)
  const InvSrc<T> isteps{loff2, linv2, nullptr, nullptr, nullptr};
  const InvSrc<T> inodes{loff2, linv2, ctx->d_ninv_off.as<int64_t>(), ctx->d_ninv_ld.as<int32_t>(),
                         ctx->d_ninv.as<T>()};
  auto one_pass = [&](int l) { return l < (int)ctx->level_one_pass.size() && ctx->level_one_pass[l]; };
  constexpr int ALL = 1 << 30;  // step length of a one-pass level
  const NodeInfo* nodes = ctx->d_nodes.as<NodeInfo>();
  const NodeState* st = ctx->d_state.as<NodeState>();
  const int32_t* lall = ctx->d_level_nodes.as<int32_t>();
  KTimer& tm = ctx->timer;
  const double sz = sizeof(T), dm = m;
  // algorithmic work of one launch over a level, with the actual pivot counts
  // algorithmic work of a level: its fronts inside the rows [rlo, rhi) (the
  // kernels take the trees outside as zero and skip them)
  const bool ranged = rlo > 0 || rhi < ctx->n;
  // the slice [q0, q1) of level l's node list (ascending starts) whose fronts lie
  // in the rows [rlo, rhi): the whole-front kernels are launched over it alone
  auto level_slice = [&](int l) {
    const int32_t* b = ctx->level_nodes.data() + ctx->level_ptr[l];
    const int nl = ctx->level_ptr[l + 1] - ctx->level_ptr[l];
    if (!ranged) return std::make_pair(0, nl);
    auto first_at = [&](int64_t r) {  // first position whose front starts at or after row r
      return (int)(std::lower_bound(b, b + nl, r, [&](int32_t j, int64_t v) { return ctx->nodes[j].start < v; }) - b);
    };
    return std::make_pair(first_at(rlo), first_at(rhi));
  };
  auto level_sum = [&](int l, auto&& fn) {
    double by = 0.0, fl = 0.0;
    if (!tm.on) return std::make_pair(by, fl);
    for (int32_t q = ctx->level_ptr[l]; q < ctx->level_ptr[l + 1]; ++q) {
      const int32_t j = ctx->level_nodes[q];
      if (ranged && (ctx->nodes[j].start < rlo || ctx->nodes[j].start >= rhi)) continue;
      fn(ctx->nodes[j], (double)ctx->hstate[j].npiv, by, fl);
    }
    return std::make_pair(by, fl);
  };
  {
    size_t need = 1;
    for (int l = 0; l < nlev; ++l) {
      const size_t nl = ctx->level_ptr[l + 1] - ctx->level_ptr[l];
      const size_t maxch = std::max<size_t>(1, cdiv(ctx->level_maxb[l], RCH));
      need = std::max(need, nl * maxch * ctx->level_maxp[l] * m);
    }
    ctx->d_part.alloc(need * sizeof(T));
  }
  // per front: the number of the last application whose gathered forward block
  // had a nonzero (written by the gathers; no clearing between applications)
  const size_t nmark = (size_t)std::max(ctx->n_nodes, 1) * sizeof(int32_t);
  if (ctx->d_live.bytes < nmark || ctx->d_tree_live.bytes < nmark || ctx->live_gen == INT32_MAX) {
    // new arrays, or all numbers used: start again from cleared ones
    ctx->d_live.alloc(nmark);
    ctx->d_tree_live.alloc(nmark);
    HF_HIP(hipMemsetAsync(ctx->d_live.ptr, 0, ctx->d_live.bytes, s));
    HF_HIP(hipMemsetAsync(ctx->d_tree_live.ptr, 0, ctx->d_tree_live.bytes, s));
    ctx->live_gen = 0;
  }
  ++ctx->live_gen;
  int32_t* live = ctx->d_live.as<int32_t>();
  const int gen = ctx->live_gen;
  const SweepMarks mk{live, ctx->d_tree_live.as<int32_t>(),
                      ctx->n_roots > 1 ? (const int32_t*)ctx->d_rootof.as<int32_t>() : nullptr, gen};
  // the backward sweep writes every row of the moderate part; the hard part's rows
  // (also read as border values) stay zero
  if (ctx->M > 0)
    k_zero_rows<<<cdiv((int64_t)ctx->M * m, 256), 256, 0, s>>>(ctx->M, m, ctx->d_l2.as<int32_t>(), Y);
  // levels whose fronts each go through one workgroup (FP32; many fronts of at
  // most one step whose backward LDS block fits)
  const int fcb = m <= 16 ? 1 : m <= 32 ? 2 : 4;
  // (forward steps of four column blocks stay level-wide: with their LDS block
  // one workgroup per CU streams the front no faster than the level launches)
  auto whole_fronts = [&](int l, bool fwd) {
    if (!std::is_same<T, float>::value || (fwd && fcb == 4)) return false;
    const int nl = ctx->level_ptr[l + 1] - ctx->level_ptr[l];
    const int mp = ctx->level_maxp[l], mb = ctx->level_maxb[l];
    const int nmin = ctx->opt.sweep_front_min;
    if (nmin <= 0 || nl < nmin || mp > TB) return false;
    return fcb == 1 ? mb + mp <= FrontBwdRows<1>::value
                    : mb <= (fcb == 2 ? FrontBwdRows<2>::value : FrontBwdRows<4>::value);
  };
  for (int l = 0; l < nlev; ++l) {
    const int nl = ctx->level_ptr[l + 1] - ctx->level_ptr[l];
    const int32_t* ln = lall + ctx->level_ptr[l];
    const int maxp = ctx->level_maxp[l], maxf = ctx->level_maxf[l];
    if constexpr (std::is_same<T, float>::value) {
      if (whole_fronts(l, true)) {
        auto wf = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
          by += np * dm * 8.0 + 0.5 * np * np * sz + ni.b * np * sz + np * dm * sz + 2.0 * ni.b * dm * sz;
          for (int32_t q = ni.child_begin; q < ni.child_end; ++q) by += ctx->nodes[ctx->child_list[q]].b * dm * sz;
          fl += dm * np * np + 2.0 * dm * ni.b * np;
        });
        const auto sl = level_slice(l);
        if (sl.second > sl.first)
        launch_timed(tm, HF_K_FWD_FRONT, wf.first, wf.second, s,
                     fcb == 1 ? k_fwd_front<1> : fcb == 2 ? k_fwd_front<2> : k_fwd_front<4>,
                     dim3((unsigned)(sl.second - sl.first)), dim3(FRONT_NT), ln + sl.first, nodes,
                     st, (const int32_t*)ctx->d_ipos.as<int32_t>(), (const int64_t*)ctx->d_gat_ptr.as<int64_t>(),
                     (const int64_t*)ctx->d_gat_src.as<int64_t>(), m, R, front, loff2, linv2, rb, zb, mk, rlo, rhi);
        continue;
      }
    }
    // the level-wide launches cover the slice of fronts inside the rows (every
    // front unless row-restricted); the choice of kernels follows the whole level
    const auto slv = level_slice(l);
    if (slv.second == slv.first) continue;
    const int nls = slv.second - slv.first;
    const int32_t* lns = ln + slv.first;
    auto wg = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
      by += ni.f * dm * sz + np * dm * 8.0;
      for (int32_t q = ni.child_begin; q < ni.child_end; ++q) {
        const double bc = ctx->nodes[ctx->child_list[q]].b;
        by += bc * dm * sz;
        fl += bc * dm;
      }
    });
    launch_timed(tm, HF_K_SOLVE_GATHER, wg.first, wg.second, s, k_fwd_gather<T>,
                 dim3(cdiv((int64_t)maxf * cdiv(m, 16), 256), nls), dim3(256), lns, nodes, st,
                 (const int32_t*)ctx->d_ipos.as<int32_t>(), (const int64_t*)ctx->d_gat_ptr.as<int64_t>(),
                 (const int64_t*)ctx->d_gat_src.as<int64_t>(), m, R, rb, mk, rlo, rhi);
    const bool op = one_pass(l);
    const int tb = op ? ALL : step_of(nl);
    const int span = op ? maxp : tb;  // rows of one diagonal product
    const InvSrc<T> inv = op ? inodes : isteps;
    for (int J0 = 0; J0 < maxp; J0 += tb) {
      auto wd = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
        if (np <= J0) return;
        const double nc = std::min<double>(tb, np - J0);
        by += 0.5 * nc * nc * sz + 2.0 * nc * dm * sz;
        fl += dm * nc * nc;
      });
      {
        dim3 g(cdiv(span, SB), nl);
        if (wide(g) && ncb > 1)
          launch_timed(tm, HF_K_FWD_DIAG, wd.first, wd.second, s,
                       op ? k_fwd_diag<T, KBW, true> : k_fwd_diag<T, KBW, false>, dim3(g.x, nls), dim3(256), lns, nodes, st, inv,
                       J0, tb, m, rb, zb, (const int32_t*)live, gen);
        else
          launch_timed(tm, HF_K_FWD_DIAG, wd.first, wd.second, s,
                       op ? pick(k_fwd_diag_n<T, 1, true>, k_fwd_diag_n<T, 2, true>, k_fwd_diag_n<T, 4, true>)
                          : pick(k_fwd_diag_n<T, 1, false>, k_fwd_diag_n<T, 2, false>, k_fwd_diag_n<T, 4, false>),
                       dim3(cdiv(span, 16), nls),
                       dim3(op ? 512 : 256), lns, nodes, st, inv, J0, tb, m, rb, zb, (const int32_t*)live, gen);
      }
      const int rows = op ? ctx->level_maxb[l] : maxf - J0 - 1;
      if (rows > 0) {
        dim3 g(cdiv(rows, 64), nl);
        auto wu = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
          if (np <= J0) return;
          const double nc = std::min<double>(tb, np - J0);
          const double below = ni.f - J0 - nc - (ni.p - np);
          if (below <= 0) return;
          by += below * nc * sz + 2.0 * below * dm * sz + nc * dm * sz;
          fl += 2.0 * dm * below * nc;
        });
        if (wide(g) && ncb > 1)
          launch_timed(tm, HF_K_FWD_UPDATE, wu.first, wu.second, s,
                       op ? k_fwd_upd<T, KBW, true> : k_fwd_upd<T, KBW, false>, dim3(g.x, nls), dim3(256), lns, nodes, st, front,
                       J0, tb, m, zb, rb, (const int32_t*)live, gen);
        else
          launch_timed(tm, HF_K_FWD_UPDATE, wu.first, wu.second, s,
                       op ? pick(k_fwd_upd_n<T, 1, true>, k_fwd_upd_n<T, 2, true>, k_fwd_upd_n<T, 4, true>)
                          : pick(k_fwd_upd_n<T, 1, false>, k_fwd_upd_n<T, 2, false>, k_fwd_upd_n<T, 4, false>),
                       dim3(cdiv(rows, 16), nls),
                       dim3(op ? 512 : 256), lns, nodes, st, front, J0, tb, m, zb, rb, (const int32_t*)live, gen);
      }
    }
  }
  for (int l = nlev - 1; l >= 0; --l) {
    const int nl = ctx->level_ptr[l + 1] - ctx->level_ptr[l];
    const int32_t* ln = lall + ctx->level_ptr[l];
    const int maxp = ctx->level_maxp[l];
    if (maxp == 0) continue;
    if constexpr (std::is_same<T, float>::value) {
      if (whole_fronts(l, false)) {
        auto wf = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
          by += ni.b * dm * 8.0 + ni.b * np * sz + np * dm * sz + np * sz + 0.5 * np * np * sz + np * dm * 8.0;
          fl += 2.0 * dm * ni.b * np + dm * np * np;
        });
        const auto sl = level_slice(l);
        if (sl.second > sl.first)
        launch_timed(tm, HF_K_BWD_FRONT, wf.first, wf.second, s,
                     fcb == 1 ? k_bwd_front<1> : fcb == 2 ? k_bwd_front<2> : k_bwd_front<4>,
                     dim3((unsigned)(sl.second - sl.first)), dim3(FRONT_NT), ln + sl.first, nodes, st, front, loff2, linv2, (const int32_t*)ctx->d_piv.as<int32_t>(),
                     (const int32_t*)ctx->d_border.as<int32_t>(), (const float*)ctx->d_dval.as<float>(), m, Y,
                     (const float*)zb, mk);
        continue;
      }
    }
    // the level-wide launches cover the slice of fronts inside the rows (every
    // front unless row-restricted); the choice of kernels follows the whole level
    const auto slv = level_slice(l);
    if (slv.second == slv.first) continue;
    const int nls = slv.second - slv.first;
    const int32_t* lns = ln + slv.first;
    const int maxch = std::max(1, (int)cdiv(ctx->level_maxb[l], RCH));
    // one chunk per front and a border on every front: the product writes t itself
    bool fused_fin = maxch == 1;
    for (int32_t q = ctx->level_ptr[l]; fused_fin && q < ctx->level_ptr[l + 1]; ++q)
      fused_fin = ctx->nodes[ctx->level_nodes[q]].b > 0;
    T* part = ctx->d_part.as<T>();
    auto wb = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
      by += ni.b * np * sz + np * dm * sz + ni.b * dm * sz;
      fl += 2.0 * dm * ni.b * np;
    });
    if (ctx->level_maxb[l] > 0) {
      auto wy = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
        by += ni.b * dm * (8.0 + sz);
      });
      timed(tm, HF_K_SOLVE_GATHER, wy.first, 0.0, s, [&] {
        dim3 gy(cdiv((int64_t)ctx->level_maxb[l] * cdiv(m, 16), 256), nls);
        k_bwd_gather<T><<<gy, 256, 0, s>>>(lns, nodes, ctx->d_border.as<int32_t>(), m, Y, rb, mk);
      });
      dim3 gp(cdiv(maxp, 64), maxch, nls);
      const T* dv = ctx->d_dval.as<T>();
      // 16 columns or fewer: the narrow form; wider blocks: 64x64 tiles staged through LDS
      dim3 gn(cdiv(maxp, 16), maxch, nls);
      if (ncb == 1)
        launch_timed(tm, HF_K_BWD_BORDER, wb.first, wb.second, s,
                     fused_fin ? k_bwd_border_n<T, 1, true> : k_bwd_border_n<T, 1, false>, gn, dim3(256), lns, nodes,
                     st, front, rb, m, maxch, maxp, part, dv, (const T*)zb, mk);
      else
        launch_timed(tm, HF_K_BWD_BORDER, wb.first, wb.second, s,
                     fused_fin ? k_bwd_border_part<T, KBN / 2, true> : k_bwd_border_part<T, KBN / 2, false>, gp,
                     dim3(256), lns, nodes, st, front, rb, m, maxch, maxp, part, dv, (const T*)zb, mk);
    }
    if (!fused_fin) {
      auto wf = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
        by += 3.0 * np * dm * sz;
      });
      timed(tm, HF_K_SOLVE_GATHER, wf.first, wf.second, s, [&] {
        dim3 gf(cdiv((int64_t)maxp * m, 256), nls);
        k_bwd_border_fin<T><<<gf, 256, 0, s>>>(lns, nodes, st, ctx->d_dval.as<T>(), m, maxch, maxp, part, zb, rb,
                                               mk);
      });
    }
    const bool op = one_pass(l);
    const int tb = op ? ALL : step_of(nl);
    const int span = op ? maxp : tb;
    const InvSrc<T> inv = op ? inodes : isteps;
    for (int J0 = ((maxp - 1) / tb) * tb; J0 >= 0; J0 -= tb) {
      auto wd = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
        if (np <= J0) return;
        const double nc = std::min<double>(tb, np - J0);
        by += 0.5 * nc * nc * sz + 2.0 * nc * dm * sz + nc * dm * 8.0;
        fl += dm * nc * nc;
      });
      {
        dim3 g(cdiv(span, SB), nl);
        if (wide(g) && ncb > 1)
          launch_timed(tm, HF_K_BWD_DIAG, wd.first, wd.second, s,
                       op ? k_bwd_diag<T, KBW, true> : k_bwd_diag<T, KBW, false>, dim3(g.x, nls), dim3(256), lns, nodes, st, inv,
                       ctx->d_piv.as<int32_t>(), J0, tb, m, Y, rb, zb, mk);
        else
          launch_timed(tm, HF_K_BWD_DIAG, wd.first, wd.second, s,
                       op ? pick(k_bwd_diag_n<T, 1, true>, k_bwd_diag_n<T, 2, true>, k_bwd_diag_n<T, 4, true>)
                          : pick(k_bwd_diag_n<T, 1, false>, k_bwd_diag_n<T, 2, false>, k_bwd_diag_n<T, 4, false>),
                       dim3(cdiv(span, 16), nls),
                       dim3(op ? 512 : 256), lns, nodes, st, inv, ctx->d_piv.as<int32_t>(), J0, tb, m, Y, rb, zb, mk);
      }
      if (J0 > 0) {
        dim3 g(cdiv(J0, 64), nl);
        auto wu = level_sum(l, [&](const NodeInfo& ni, double np, double& by, double& fl) {
          if (np <= J0) return;
          const double nc = std::min<double>(tb, np - J0);
          by += J0 * nc * sz + 2.0 * J0 * dm * sz;
          fl += 2.0 * dm * J0 * nc;
        });
        if (wide(g) && ncb > 1)
          launch_timed(tm, HF_K_BWD_UPDATE, wu.first, wu.second, s, k_bwd_upd<T, KBW>, dim3(g.x, nls), dim3(256), lns, nodes, st,
                       front, J0, tb, m, zb, rb, mk);
        else
          launch_timed(tm, HF_K_BWD_UPDATE, wu.first, wu.second, s,
                       pick(k_bwd_upd_n<T, 1>, k_bwd_upd_n<T, 2>, k_bwd_upd_n<T, 4>), dim3(cdiv(J0, 16), nls),
                       dim3(256), lns, nodes, st, front, J0, tb, m, zb, rb, mk);
      }
    }
  }
  HF_HIP(hipGetLastError());
}

template void step_inverses<float>(hf_ctx*, int, hipStream_t);
template void step_inverses<double>(hf_ctx*, int, hipStream_t);
template void node_inverses<float>(hf_ctx*, hipStream_t);
template void node_inverses<double>(hf_ctx*, hipStream_t);
template void precond_apply<float>(hf_ctx*, int, const double*, double*, hipStream_t, int64_t, int64_t);
template void precond_apply<double>(hf_ctx*, int, const double*, double*, hipStream_t, int64_t, int64_t);

}  // namespace hf
