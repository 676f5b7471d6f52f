// FP64 part of the hybrid factorization on the GPU.
//
//   - CSR SpMM with the moderate / hard masks (A = K11 of Algorithm 1 step 2)
//   - tall-skinny Gram products with a fixed-order two-stage reduction
//   - small dense kernels: pivoted Cholesky with deflation of the block-GCR
//     Gram matrices, coefficient solves, block combinations
//   - Algorithm 5 (preconditioned block GCR) driven from the host, one small
//     device-to-host read of the residual norms per iteration
//   - Algorithm 1 steps 2-5: K12 blocks, X12, S22 = K22 - K21 X12, the FP64
//     rank-revealing LDL^T of S22 (1x1 / 2x2 symmetric pivoting), kernel lift
//   - Algorithm 2 (solve)
// All vectors are row-major n x m (m right-hand sides contiguous per row) in
// elimination order unless stated otherwise.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <type_traits>

#include <hip/hip_cooperative_groups.h>

#include "hf_internal.h"
#include "hf_kernels.h"

namespace hf {

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

constexpr int GRAM_WG = 256;   // partial sums of a Gram product (fixed: reduction order)
constexpr int MAXM = 64;       // widest block handled by the small dense kernels
// The kernel basis (n x k) is stored as column chunks of KC columns, chunk c a
// row-major n x min(KC, k - c KC) block at offset c n KC, so every dense product
// with it stays within the small kernels' width.
constexpr int KC = MAXM;
constexpr int KMAX = 1024;     // largest kernel dimension handled
constexpr int S22_GRID_MAXM = 2048;  // largest S22 factorized over a cooperative grid
constexpr int S22_LDS_M = 8192;  // S22 solves keep their work column (M doubles) in LDS up to this M
static inline int kchunk(int k, int c) { return std::min(KC, k - c * KC); }

// ---------------------------------------------------------------------------
// SpMM and friends
// ---------------------------------------------------------------------------

// Y = K11 W (rows and columns of the hard part masked out); one thread per (row,
// pair of columns), the pair moved in 16-byte pieces
__global__ void k_spmm_k11(int64_t row0, int64_t row1, const int64_t* __restrict__ ip,
                           const int32_t* __restrict__ ix, const double* __restrict__ kv,
                           const uint8_t* __restrict__ isl2, int m, const double* __restrict__ W,
                           double* __restrict__ Y) {
  const int mh = (m + 1) >> 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rr = e / mh;
  const int col = 2 * (int)(e - rr * mh);
  const int64_t row = row0 + rr;
  if (row >= row1) return;
  const bool two = col + 1 < m;
  double acc0 = 0.0, acc1 = 0.0;
  if (!isl2[row]) {
    const int64_t q1 = ip[row + 1];
    for (int64_t q0 = ip[row]; q0 < q1; q0 += 8) {  // eight entries' loads in flight, summed in order
      double a[8], w0[8], w1[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a[i] = 0.0;
        w0[i] = 0.0;
        w1[i] = 0.0;
        if (q0 + i < q1) {
          const int32_t c = ix[q0 + i];
          if (!isl2[c]) {
            a[i] = kv[q0 + i];
            const double* src = W + (int64_t)c * m + col;
            if (two) {
              double x[2];
              __builtin_memcpy(x, src, 16);
              w0[i] = x[0];
              w1[i] = x[1];
            } else {
              w0[i] = src[0];
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (q0 + i < q1) {
          acc0 += a[i] * w0[i];
          acc1 += a[i] * w1[i];
        }
    }
  }
  double* dst = Y + row * m + col;
  dst[0] = acc0;
  if (two) dst[1] = acc1;
}

// Residual of the caller's system, returned scaled and in elimination order:
// r_g = q_g (bbar_{perm g} - sum_e Kbar_e xo_{perm c_e}), xo being the current
// solution in the caller's variables (row-major n x m, original order) and B the
// caller's column-major right-hand side block (columns c0.., leading dimension ldb).
// The sum is carried in double-double: every product is split exactly into a
// rounded part and its error (fused multiply-add) and every addition into its
// sum and error (two-sum), the errors being accumulated on the side (compensated
// dot product of Ogita, Rump and Oishi).  The residual is then accurate to a few
// units of its own size, not of |Kbar| |xo|, so a correction pass can reduce the
// forward error below the conditioning limit of an FP64 residual.
__global__ void k_residual_orig(int64_t n, const int64_t* __restrict__ ip, const int32_t* __restrict__ ix,
                                const double* __restrict__ kbar, const double* __restrict__ qp,
                                const int32_t* __restrict__ perm, int m, const double* __restrict__ B,
                                int64_t ldb, int c0, const double* __restrict__ xo, double* __restrict__ R) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = e / m;
  const int col = (int)(e - row * m);
  if (row >= n) return;
  double sh = B[(int64_t)(c0 + col) * ldb + perm[row]], sl = 0.0;
  for (int64_t q = ip[row]; q < ip[row + 1]; ++q) {
    const double a = kbar[q], x = xo[(int64_t)perm[ix[q]] * m + col];
    const double p = a * x;
    const double pe = fma(a, x, -p);  // a x = p + pe exactly
    const double t = sh - p;          // sh - p = t + te exactly
    const double z = t - sh;
    const double te = (sh - (t - z)) - (p + z);
    sh = t;
    sl += te - pe;
  }
  R[e] = qp[row] * (sh + sl);
}

__global__ void k_add(int64_t nm, double* __restrict__ x, const double* __restrict__ d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nm) x[e] += d[e];
}

// out = B - Y   (elementwise, n*m)
__global__ void k_sub(int64_t nm, const double* __restrict__ B, const double* __restrict__ Y,
                      double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nm) out[e] = B[e] - Y[e];
}

// K12 column block: B[g, c] = K[g, l2[c0+c]] for g in the moderate part, 0 else.
__global__ void k_gather_k12(const int64_t* __restrict__ ip, const int32_t* __restrict__ ix,
                             const double* __restrict__ kv, const uint8_t* __restrict__ isl2,
                             const int32_t* __restrict__ l2, int c0, int nbc, int mb,
                             double* __restrict__ B) {
  const int c = blockIdx.x;
  if (c >= nbc) return;
  const int32_t x = l2[c0 + c];
  for (int64_t q = ip[x] + threadIdx.x; q < ip[x + 1]; q += blockDim.x) {
    const int32_t g = ix[q];
    if (!isl2[g]) B[(int64_t)g * mb + c] = kv[q];  // K symmetric: K[g, x] = K[x, g]
  }
}

// S22 column block: S[i, c0+c] = sum_q K[l2_i, x_q] W[x_q, c], W = [-X12; I].
__global__ void k_s22_block(const int64_t* __restrict__ ip, const int32_t* __restrict__ ix,
                            const double* __restrict__ kv, const uint8_t* __restrict__ isl2,
                            const int32_t* __restrict__ l2, int M, int c0, int nbc, int mb,
                            const double* __restrict__ Xb, double* __restrict__ S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / nbc, c = e - (e / nbc) * nbc;
  if (i >= M) return;
  const int32_t g = l2[i];
  const int32_t target = l2[c0 + c];
  double acc = 0.0;
  for (int64_t q = ip[g]; q < ip[g + 1]; ++q) {
    const int32_t x = ix[q];
    if (isl2[x]) {
      if (x == target) acc += kv[q];
    } else {
      acc -= kv[q] * Xb[(int64_t)x * mb + c];
    }
  }
  S[(int64_t)(c0 + c) * M + i] = acc;
}

__global__ void k_symmetrize(int M, double* __restrict__ S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / M, j = e - (e / M) * M;
  if (i >= M || j >= i) return;
  const double a = 0.5 * (S[(int64_t)j * M + i] + S[(int64_t)i * M + j]);
  S[(int64_t)j * M + i] = a;
  S[(int64_t)i * M + j] = a;
}

// y2[i, c] = b[l2_i, c] - sum_{x moderate} K[l2_i, x] y1[x, c]
__global__ void k_y2(const int64_t* __restrict__ ip, const int32_t* __restrict__ ix,
                     const double* __restrict__ kv, const uint8_t* __restrict__ isl2,
                     const int32_t* __restrict__ l2, int M, int m, const double* __restrict__ b,
                     const double* __restrict__ y1, double* __restrict__ y2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / m, c = e - (e / m) * m;
  if (i >= M) return;
  const int32_t g = l2[i];
  double acc = b[(int64_t)g * m + c];
  for (int64_t q = ip[g]; q < ip[g + 1]; ++q) {
    const int32_t x = ix[q];
    if (!isl2[x]) acc -= kv[q] * y1[(int64_t)x * m + c];
  }
  y2[(int64_t)i * m + c] = acc;
}

// ---------------------------------------------------------------------------
// Gram products C = A^T B (A: n x a, B: n x b, row-major), fixed-order sums
// ---------------------------------------------------------------------------

// One 64 x 64 (a x b) partial Gram tile per workgroup over a fixed row range,
// FP64 matrix cores; k_gram_reduce sums the GRAM_WG partials in a fixed order.
constexpr int GLD = 68;
constexpr int GKB = 64;  // k per stage of the Gram tiles
constexpr int CKB = 16;  // k per stage of the combine tiles: small stages, several workgroups per CU
__global__ void __launch_bounds__(256)
k_gram_partial(int64_t n, int a, const double* __restrict__ A, int64_t sA, int b,
               const double* __restrict__ B, double* __restrict__ partial) {
  const int blk = blockIdx.y;
  const double* Ab = A + (int64_t)blk * sA;
  const int64_t chunk = (n + GRAM_WG - 1) / GRAM_WG;
  const int r0 = (int)((int64_t)blockIdx.x * chunk);
  const int r1 = (int)min(n, (int64_t)r0 + chunk);
  __shared__ double As[GKB][GLD];
  __shared__ double Bs[GKB][GLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  Mfma<double>::V acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<double>::V{0, 0, 0, 0};
  tile_gemm_64<double, GKB, GLD, false>(
      acc, As, Bs, r0, r1, [&](int k, int i) { return i < a ? Ab[(int64_t)k * a + i] : 0.0; },
      [&](int k, int j) { return j < b ? B[(int64_t)k * b + j] : 0.0; }, tid, lane, wr, wc);
  double* out = partial + ((int64_t)blk * GRAM_WG + blockIdx.x) * a * b;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = wr + bi * 16 + Mfma<double>::row(lane, t), j = wc + bj * 16 + (lane & 15);
        if (i < a && j < b) out[i * b + j] = acc[bi][bj][t];
      }
}

// Squared column norms of an n x m row-major block (the convergence test needs
// only the diagonal of R^T R): GRAM_WG row chunks, each summed by 4 row phases
// of 64 columns and the phases added in order; k_colsq_reduce adds the chunks
// in order.
__global__ void __launch_bounds__(256)
k_colsq_partial(int64_t n, int m, const double* __restrict__ R, double* __restrict__ partial) {
  const int64_t chunk = (n + GRAM_WG - 1) / GRAM_WG;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  __shared__ double red[4][64];
  double acc = 0.0;
  if (c < m)
    for (int64_t r = r0 + ph; r < r1; r += 32) {  // eight rows of this phase in flight
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (r + 4 * i < r1) ? R[(r + 4 * i) * m + c] : 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += v[i] * v[i];
    }
  red[ph][c] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && c < m)
    partial[(int64_t)blockIdx.x * m + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// Fixed-order sums of GRAM_WG partials (bitwise reproducible): 1024 threads per
// 64 consecutive entries; wave ph adds partials ph, ph + 16, ph + 32, ... in
// order, then the 16 wave sums are added in order.
constexpr int RED_WAVES = 16;
__device__ __forceinline__ double fixed_order_sum(const double* __restrict__ P, int64_t stride, bool ok) {
  __shared__ double red[RED_WAVES][64];
  const int lane = threadIdx.x & 63, ph = threadIdx.x >> 6;
  double s = 0.0;
  if (ok)
    for (int w = ph; w < GRAM_WG; w += RED_WAVES) s += P[(int64_t)w * stride];
  red[ph][lane] = s;
  __syncthreads();
  double t = 0.0;
  if (ph == 0)
    for (int q = 0; q < RED_WAVES; ++q) t += red[q][lane];
  return t;
}

__global__ void __launch_bounds__(1024) k_colsq_reduce(int m, const double* __restrict__ partial,
                                                       double* __restrict__ out) {
  const int c = threadIdx.x & 63;
  const double s = fixed_order_sum(partial + c, m, c < m);
  if ((threadIdx.x >> 6) == 0 && c < m) out[c] = s;
}

__global__ void __launch_bounds__(1024) k_gram_reduce(int nblk, int ab, const double* __restrict__ partial,
                                                      double* __restrict__ out) {
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  const bool ok = e < nblk * ab;
  const int blk = ok ? e / ab : 0, pidx = ok ? e - blk * ab : 0;
  const double s = fixed_order_sum(partial + (int64_t)blk * GRAM_WG * ab + pidx, ab, ok);
  if ((threadIdx.x >> 6) == 0 && ok) out[e] = s;
}

// ---------------------------------------------------------------------------
// small dense FP64 kernels (one workgroup per matrix)
// ---------------------------------------------------------------------------

// value of lane t (wave-uniform t) in every lane, through scalar registers
__device__ __forceinline__ double lane_bcast(double v, int t) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), t);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), t);
  return __hiloint2double(hi, lo);
}

// Pivoted Cholesky of an SPSD m x m Gram matrix (row-major), deflating pivots
// <= rel * max diag.  Output: Lc (m x m row-major, lower), piv[m], rank.
// Four waves: every wave finds the pivot itself (lanes over the diagonal), the
// trailing update runs with waves over rows and lanes over columns.
__global__ void __launch_bounds__(256)
k_chol_piv(int m, const double* __restrict__ Mm, int64_t sM, double* __restrict__ Lc,
           int32_t* __restrict__ piv, int32_t* __restrict__ rank, double rel) {
  const int blk = blockIdx.x;
  const double* G = Mm + (int64_t)blk * sM;
  double* Lg = Lc + (int64_t)blk * m * m;
  int32_t* P = piv + (int64_t)blk * m;
  __shared__ double A[MAXM * MAXM];
  __shared__ double L[MAXM * MAXM];
  __shared__ double Lt[MAXM * MAXM];  // column i of L for the trailing update, lanes consecutive
  __shared__ int Ps[MAXM];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < m * m; e += 256) { A[e] = G[e]; L[e] = 0.0; }
  for (int e = tid; e < m; e += 256) Ps[e] = e;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < m; ++i) dmax = fmax(dmax, A[i * m + i]);
  int i;
  for (i = 0; i < m; ++i) {
    // largest remaining diagonal, ties to the first
    double bv = -INFINITY;
    int bk = INT_MAX;
    if (lane >= i && lane < m) { bv = A[lane * m + lane]; bk = lane; }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int ok = __shfl_xor(bk, off, 64);
      if (ov > bv || (ov == bv && ok < bk)) { bv = ov; bk = ok; }
    }
    const int k = bk;
    if (bv <= rel * dmax || bv <= 0.0) break;
    if (k != i) {
      for (int t = tid; t < m; t += 256) {
        const double x = A[i * m + t]; A[i * m + t] = A[k * m + t]; A[k * m + t] = x;
      }
      __syncthreads();
      for (int t = tid; t < m; t += 256) {
        const double x = A[t * m + i]; A[t * m + i] = A[t * m + k]; A[t * m + k] = x;
      }
      for (int t = tid; t < i; t += 256) {
        const double x = L[i * m + t]; L[i * m + t] = L[k * m + t]; L[k * m + t] = x;
      }
      if (tid == 0) { const int x = Ps[i]; Ps[i] = Ps[k]; Ps[k] = x; }
      __syncthreads();
    }
    const double lii = sqrt(A[i * m + i]);
    for (int r = i + tid; r < m; r += 256) {
      const double x = (r == i) ? lii : A[r * m + i] / lii;
      L[r * m + i] = x;
      Lt[i * m + r] = x;
    }
    __syncthreads();
    const int c = i + 1 + lane;
    if (c < m)
      for (int r = i + 1 + w; r < m; r += 4) A[r * m + c] -= L[r * m + i] * Lt[i * m + c];
    __syncthreads();
  }
  for (int e = tid; e < m * m; e += 256) Lg[e] = L[e];
  for (int e = tid; e < m; e += 256) P[e] = Ps[e];
  if (tid == 0) rank[blk] = i;
}

// out = sign * M^{-1} R for every batch item (R: m x nc row-major), deflated
// directions get 0.  One workgroup per batch item; each wave takes columns of R
// in turn and holds one column in its lanes (lane i: row i), so the two
// triangular sweeps are lane-parallel: after row t is final it is broadcast and
// every later row subtracts its multiple (for row i the forward subtractions
// run in the same order t = 0 .. i-1 as a row-by-row substitution).
__global__ void __launch_bounds__(1024)
k_chol_solve(int m, int nc, const double* __restrict__ Lc, const int32_t* __restrict__ piv,
             const int32_t* __restrict__ rank, const double* __restrict__ R,
             int64_t sR, double* __restrict__ out, int64_t sO, double sign) {
  const int blk = blockIdx.x;
  const double* Lg = Lc + (int64_t)blk * m * m;
  const int32_t* P = piv + (int64_t)blk * m;
  __shared__ double L[MAXM * MAXM];   // row-major, as in global memory
  __shared__ double Lt[MAXM * MAXM];  // its transpose: lanes read consecutive words
  __shared__ int Ps[MAXM];
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const double x = Lg[e];
    L[e] = x;
    Lt[(e % m) * m + e / m] = x;
  }
  for (int e = threadIdx.x; e < m; e += blockDim.x) Ps[e] = P[e];
  __syncthreads();
  const int rk = rank[blk];
  const double* Rb = R + (int64_t)blk * sR;
  double* O = out + (int64_t)blk * sO;
  const int i = threadIdx.x & 63, nw = blockDim.x >> 6;
  const double lii = (i < rk) ? L[i * m + i] : 1.0;
  for (int c = threadIdx.x >> 6; c < nc; c += nw) {
    double z = (i < rk) ? Rb[(int64_t)Ps[i] * nc + c] : 0.0;
    // forward: L z = R
    for (int t = 0; t < rk; ++t) {
      if (i == t) z = z / lii;
      const double zt = lane_bcast(z, t);
      if (i > t && i < rk) z -= Lt[t * m + i] * zt;
    }
    // backward: L^T z = z
    for (int t = rk - 1; t >= 0; --t) {
      if (i == t) z = z / lii;
      const double zt = lane_bcast(z, t);
      if (i < t) z -= L[t * m + i] * zt;
    }
    if (i < m) O[(int64_t)Ps[i] * nc + c] = (i < rk) ? sign * z : 0.0;
  }
}

// out[row, col] = (base ? base[row, col] : 0) + sum_t sum_k V_t[row, k] coef_t[k, col]
// V_t = V + t*sV (n x a, row-major), coef_t = coef + t*a*b (a x b), out n x b.
// out (n x b) = base + sum_t V_t (n x a) C_t (a x b); V_t = V + t sV and C_t
// = coef + t a b, all row-major; base may alias out or be null.  One 64-row
// strip per workgroup, the nterms products concatenated along k (FP64 matrix
// cores).
__global__ void __launch_bounds__(256)
k_combine(int64_t n, int a, int b, double* out, const double* base, int nterms,
          const double* __restrict__ V, int64_t sV, const double* __restrict__ coef,
          const int64_t* __restrict__ rng) {
  constexpr int NE = CKB * 64 / 256;
  const int r0 = blockIdx.x * 64;
  const int nrows = (int)min((int64_t)64, n - r0);
  __shared__ double As[CKB][GLD];
  __shared__ double Bs[CKB][GLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int K = a * nterms;
  Mfma<double>::V acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<double>::V{0, 0, 0, 0};
  // with rng (a a multiple of CKB), term t holds zeros outside rows
  // [rng[2t], rng[2t+1]): its stages are skipped on tiles outside them, which
  // leaves out exact zero products only
  auto next = [&](int k0) {
    if (rng)
      while (k0 < K) {
        const int t = k0 / a;
        if (r0 + 64 > rng[2 * t] && r0 < rng[2 * t + 1]) break;
        k0 += CKB;
      }
    return k0;
  };
  double ra[NE], rb[NE];
  auto fetch = [&](int k0) {  // A contiguous in k
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + 256 * q;
      const int kq = e % CKB, row = e / CKB;
      const int k = k0 + kq, t = k / a, kk = k - t * a;
      ra[q] = (k < K && row < nrows) ? V[t * sV + (int64_t)(r0 + row) * a + kk] : 0.0;
      const int kb = k0 + (e >> 6), col = e & 63;
      const int tb = kb / a, kkb = kb - tb * a;
      rb[q] = (kb < K && col < b) ? coef[((int64_t)tb * a + kkb) * b + col] : 0.0;
    }
  };
  int k0 = next(0);
  if (k0 < K) fetch(k0);
  while (k0 < K) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = tid + 256 * q;
      As[e % CKB][e / CKB] = ra[q];
      Bs[e >> 6][e & 63] = rb[q];
    }
    __syncthreads();
    const int k1 = next(k0 + CKB);
    if (k1 < K) fetch(k1);
    mfma_tile_64<double, CKB, GLD>(As, Bs, acc, lane, wr, wc);
    __syncthreads();
    k0 = k1;
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = wr + bi * 16 + Mfma<double>::row(lane, t), c = wc + bj * 16 + (lane & 15);
        if (r < nrows && c < b) {
          const int64_t e = (int64_t)(r0 + r) * b + c;
          out[e] = (base ? base[e] : 0.0) + acc[bi][bj][t];
        }
      }
}

// ---------------------------------------------------------------------------
// Algorithm 1 step 5: FP64 LDL^T of S22 with complete (Bunch-Parlett) pivoting,
// second-stage postponing, enlargement and the kernel decision.  One workgroup.
// A (M x M, col-major, destroyed), L (M x M col-major, unit lower), D (M x M),
// perm[M], mags[M]; info: [0] k, [1] postponed, [2] candidates, [3] gap (double).
// ---------------------------------------------------------------------------

__device__ inline double& at(double* A, int M, int r, int c) { return A[(int64_t)c * M + r]; }

constexpr int S22_NT = 1024;  // threads of the S22 factorization (16 waves)

__global__ void __launch_bounds__(S22_NT)
k_s22_ldlt(int M, double* __restrict__ Ag, double* __restrict__ L, double* __restrict__ D,
           int32_t* __restrict__ perm, double* __restrict__ mags, int32_t* __restrict__ bsize,
           double tau, int n_enlarge, double ker_tol, double* __restrict__ info) {
  constexpr int NT = S22_NT, NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  __shared__ double rv[NW];
  __shared__ int rk[NW];
  __shared__ double sA[MAXM * MAXM];  // the working copy stays in LDS when it fits
  double* A = (M <= MAXM) ? sA : Ag;
  // otherwise LDS holds the step's column(s) of L, read by every trailing column
  const bool stage = M > MAXM && 2 * M <= MAXM * MAXM;
  if (M <= MAXM)
    for (int e = tid; e < M * M; e += NT) sA[e] = Ag[e];
  // workgroup argmax of (v, k): largest v, ties to the smallest k; uniform result
  auto argmax = [&](double& v, int& k) {
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int ok = __shfl_xor(k, off, 64);
      if (ov > v || (ov == v && ok < k)) { v = ov; k = ok; }
    }
    __syncthreads();  // rv/rk free
    if (lane == 0) { rv[wv] = v; rk[wv] = k; }
    __syncthreads();
    v = rv[0];
    k = rk[0];
    for (int w = 1; w < NW; ++w)
      if (rv[w] > v || (rv[w] == v && rk[w] < k)) { v = rv[w]; k = rk[w]; }
  };
  for (int64_t e = tid; e < (int64_t)M * M; e += NT) {
    const int r = (int)(e % M), c = (int)(e / M);
    L[e] = (r == c) ? 1.0 : 0.0;
    D[e] = 0.0;
  }
  for (int e = tid; e < M; e += NT) { perm[e] = e; mags[e] = 0.0; bsize[e] = 1; }
  __syncthreads();
  auto swap = [&](int i, int k) {
    if (i == k) return;
    for (int t = tid; t < M; t += NT) { const double x = at(A, M, i, t); at(A, M, i, t) = at(A, M, k, t); at(A, M, k, t) = x; }
    __syncthreads();
    for (int t = tid; t < M; t += NT) { const double x = at(A, M, t, i); at(A, M, t, i) = at(A, M, t, k); at(A, M, t, k) = x; }
    for (int t = tid; t < i; t += NT) { const double x = at(L, M, i, t); at(L, M, i, t) = at(L, M, k, t); at(L, M, k, t) = x; }
    if (tid == 0) { const int32_t x = perm[i]; perm[i] = perm[k]; perm[k] = x; }
    __syncthreads();
  };
  // candidates of the trailing block starting at i0, gathered by this thread:
  // largest |diagonal| (position t, first occurrence) and largest |off-diagonal|
  // of the upper triangle (row-major index e over the block, first occurrence).
  // The trailing update of a step produces them for the next step's block as it
  // writes it, so the block is not read a second time.
  double bv = -1.0, ov = -1.0;
  int bk = INT_MAX, ok = INT_MAX;
  auto consider = [&](int i0, int r, int c, double v) {
    const int w = M - i0, rr = r - i0, cc = c - i0;
    const double x = fabs(v);
    if (rr == cc) {
      if (x > bv || (x == bv && rr < bk)) { bv = x; bk = rr; }
    } else if (rr < cc) {
      const int e = rr * w + cc;
      if (x > ov || (x == ov && e < ok)) { ov = x; ok = e; }
    }
  };
  for (int c = wv; c < M; c += NW)  // the first block: read once
    for (int r = lane; r <= c; r += 64) consider(0, r, c, at(A, M, r, c));
  int i = 0;
  while (i < M) {
    const int w = M - i;
    argmax(bv, bk);
    const double gd = bv;
    const int kd = bk;
    argmax(ov, ok);
    const double go = (w > 1) ? ov : 0.0;
    const int s_r = (w > 1) ? ok / w : 0;
    const int s_c = (w > 1) ? ok % w : 0;
    bv = -1.0; ov = -1.0; bk = INT_MAX; ok = INT_MAX;  // this step's update gathers the next block's
    int mode;
    if (gd == 0.0 && go == 0.0) mode = 0;
    else if (gd >= alpha * go) mode = 1;
    else mode = 2;
    if (mode == 0) break;  // exactly zero remainder: zero pivots
    if (mode == 1) {
      swap(i, i + kd);
      const double d = at(A, M, i, i);
      at(D, M, i, i) = d;
      for (int r = i + 1 + tid; r < M; r += NT) {
        const double l = at(A, M, r, i) / d;
        at(L, M, r, i) = l;
        if (stage) sA[r] = l;
      }
      __syncthreads();
      const double* li = stage ? sA : L + (int64_t)i * M;  // li[r] = L(r, i)
      for (int c = i + 1 + wv; c < M; c += NW) {
        const double aic = at(A, M, i, c);
        double* Ac = A + (int64_t)c * M;
        int r = i + 1 + lane;
        for (; r + 192 < M; r += 256) {  // four rows per lane in flight
          const double a0 = Ac[r], a1 = Ac[r + 64], a2 = Ac[r + 128], a3 = Ac[r + 192];
          const double v0 = a0 - li[r] * aic, v1 = a1 - li[r + 64] * aic;
          const double v2 = a2 - li[r + 128] * aic, v3 = a3 - li[r + 192] * aic;
          Ac[r] = v0; Ac[r + 64] = v1; Ac[r + 128] = v2; Ac[r + 192] = v3;
          consider(i + 1, r, c, v0); consider(i + 1, r + 64, c, v1);
          consider(i + 1, r + 128, c, v2); consider(i + 1, r + 192, c, v3);
        }
        for (; r < M; r += 64) {
          const double v = Ac[r] - li[r] * aic;
          Ac[r] = v;
          consider(i + 1, r, c, v);
        }
      }
      __syncthreads();
      for (int r = i + 1 + tid; r < M; r += NT) { at(A, M, r, i) = 0.0; at(A, M, i, r) = 0.0; }
      if (tid == 0) mags[i] = fabs(d);
      __syncthreads();
      i += 1;
    } else {
      const int r = s_r, c = s_c;
      swap(i, i + r);
      swap(i + 1, i + c);
      const double e11 = at(A, M, i, i), e12 = at(A, M, i + 1, i), e22 = at(A, M, i + 1, i + 1);
      const double det = e11 * e22 - e12 * e12;
      // Lc = C E^{-1}, C = A[i+2:, i:i+2]
      for (int rr = i + 2 + tid; rr < M; rr += NT) {
        const double c1 = at(A, M, rr, i), c2 = at(A, M, rr, i + 1);
        const double l0 = (c1 * e22 - c2 * e12) / det, l1 = (c2 * e11 - c1 * e12) / det;
        at(L, M, rr, i) = l0;
        at(L, M, rr, i + 1) = l1;
        if (stage) { sA[rr] = l0; sA[M + rr] = l1; }
      }
      __syncthreads();
      const double* l0s = stage ? sA : L + (int64_t)i * M;  // L(rr, i), L(rr, i+1)
      const double* l1s = stage ? sA + M : L + (int64_t)(i + 1) * M;
      for (int cc = i + 2 + wv; cc < M; cc += NW) {
        const double b0 = at(A, M, cc, i), b1 = at(A, M, cc, i + 1);
        double* Ac = A + (int64_t)cc * M;
        int rr = i + 2 + lane;
        for (; rr + 192 < M; rr += 256) {
          const double a0 = Ac[rr], a1 = Ac[rr + 64], a2 = Ac[rr + 128], a3 = Ac[rr + 192];
          const double v0 = a0 - (l0s[rr] * b0 + l1s[rr] * b1);
          const double v1 = a1 - (l0s[rr + 64] * b0 + l1s[rr + 64] * b1);
          const double v2 = a2 - (l0s[rr + 128] * b0 + l1s[rr + 128] * b1);
          const double v3 = a3 - (l0s[rr + 192] * b0 + l1s[rr + 192] * b1);
          Ac[rr] = v0; Ac[rr + 64] = v1; Ac[rr + 128] = v2; Ac[rr + 192] = v3;
          consider(i + 2, rr, cc, v0); consider(i + 2, rr + 64, cc, v1);
          consider(i + 2, rr + 128, cc, v2); consider(i + 2, rr + 192, cc, v3);
        }
        for (; rr < M; rr += 64) {
          const double v = Ac[rr] - (l0s[rr] * b0 + l1s[rr] * b1);
          Ac[rr] = v;
          consider(i + 2, rr, cc, v);
        }
      }
      __syncthreads();
      for (int rr = i + 2 + tid; rr < M; rr += NT) {
        at(A, M, rr, i) = 0.0; at(A, M, i, rr) = 0.0;
        at(A, M, rr, i + 1) = 0.0; at(A, M, i + 1, rr) = 0.0;
      }
      if (tid == 0) {
        at(D, M, i, i) = e11; at(D, M, i + 1, i) = e12; at(D, M, i, i + 1) = e12; at(D, M, i + 1, i + 1) = e22;
        const double h = 0.5 * (e11 + e22), q = sqrt(0.25 * (e11 - e22) * (e11 - e22) + e12 * e12);
        const double mg = fmin(fabs(h - q), fabs(h + q));
        mags[i] = mg; mags[i + 1] = mg;
        bsize[i] = 2; bsize[i + 1] = 0;
      }
      __syncthreads();
      i += 2;
    }
  }
  // rank decision (same rule as the oracle)
  if (tid == 0) {
    // second-stage postponing: the first pivot is compared with 1 (unit diagonal
    // of the scaled matrix), later ones with their predecessor
    int t = M;
    double prev = 1.0;
    for (int q = 0; q < M; ++q) {
      if (mags[q] == 0.0 || mags[q] < tau * prev) { t = q; break; }
      prev = mags[q];
    }
    const int postponed = M - t;
    const int e = postponed > 0 ? min(n_enlarge, t) : 0;
    int start = t - e;
    // a 2x2 block is one pivot: the candidates start at a block boundary, so the
    // kernel count (and the rank M - k) never splits a block
    if (start > 0 && start < M && bsize[start] == 0) --start;
    int k = 0;
    for (int q = M - 1; q >= start; --q) {
      if (mags[q] <= ker_tol) ++k;
      else break;
    }
    double gap = INFINITY;
    if (k > 0 && start < M - k) {
      double mn = INFINITY, mx = 0.0;
      for (int q = start; q < M - k; ++q) mn = fmin(mn, mags[q]);
      for (int q = M - k; q < M; ++q) mx = fmax(mx, mags[q]);
      gap = mn / fmax(mx, 1e-300);
    }
    info[0] = k;
    info[1] = postponed;
    info[2] = M - start;
    info[3] = gap;
  }
}

// The same factorization over the workgroups of a cooperative grid, for
// MAXM < M <= S22_GRID_MAXM.  No row or column moves: the pivots are eliminated
// where they stand, and perm (position -> original index) with its inverse pos
// replays the interchanges, so the search breaks ties on the same positions and
// every entry of the trailing block goes through the same operations as above.
// Workgroup g updates the columns b = g (mod G); each workgroup publishes the
// best candidates of its columns in a slot (two sets, alternating by step) and
// one grid barrier per step separates an update from the next search.  Lo
// receives L by original row (column j: step j); k_s22_lorder puts its rows in
// position order.
struct S22Cand {
  double dv, ov;
  int dk, ok;
};

__global__ void __launch_bounds__(S22_NT)
k_s22_ldlt_grid(int M, double* __restrict__ A, double* __restrict__ Lo, double* __restrict__ D,
                int32_t* __restrict__ perm_out, double* __restrict__ mags, int32_t* __restrict__ bsize, double tau,
                int n_enlarge, double ker_tol, double* __restrict__ info, S22Cand* __restrict__ slots) {
  constexpr int NT = S22_NT, NW = NT / 64;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  extern __shared__ double dsm[];
  double* l0 = dsm;      // the step's column(s) of L by original row
  double* l1 = dsm + M;
  int32_t* perm = reinterpret_cast<int32_t*>(dsm + 2 * M);
  int32_t* pos = perm + M;
  __shared__ double rv[2][NW];
  __shared__ int rk[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = blockIdx.x, G = gridDim.x;
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  // workgroup argmax of both candidate pairs at once (largest value, ties to the
  // smallest index); uniform result
  auto argmax2 = [&](double& v, int& k, double& u, int& m) {
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64), ou = __shfl_xor(u, off, 64);
      const int ok = __shfl_xor(k, off, 64), om = __shfl_xor(m, off, 64);
      if (ov > v || (ov == v && ok < k)) { v = ov; k = ok; }
      if (ou > u || (ou == u && om < m)) { u = ou; m = om; }
    }
    __syncthreads();
    if (lane == 0) { rv[0][wv] = v; rk[0][wv] = k; rv[1][wv] = u; rk[1][wv] = m; }
    __syncthreads();
    v = rv[0][0]; k = rk[0][0]; u = rv[1][0]; m = rk[1][0];
    for (int w = 1; w < NW; ++w) {
      if (rv[0][w] > v || (rv[0][w] == v && rk[0][w] < k)) { v = rv[0][w]; k = rk[0][w]; }
      if (rv[1][w] > u || (rv[1][w] == u && rk[1][w] < m)) { u = rv[1][w]; m = rk[1][w]; }
    }
  };
  for (int e = tid; e < M; e += NT) { perm[e] = e; pos[e] = e; }
  for (int64_t e = (int64_t)g * NT + tid; e < (int64_t)M * M; e += (int64_t)G * NT) { Lo[e] = 0.0; D[e] = 0.0; }
  if (g == 0)
    for (int e = tid; e < M; e += NT) { mags[e] = 0.0; bsize[e] = 1; }
  double bv = -1.0, ov = -1.0;
  int bk = INT_MAX, ok = INT_MAX;
  auto consider = [&](int i0, int rr, int cc, double v) {  // positions relative to i0
    const int w = M - i0;
    const double x = fabs(v);
    if (rr == cc) {
      if (x > bv || (x == bv && rr < bk)) { bv = x; bk = rr; }
    } else if (rr < cc) {
      const int e = rr * w + cc;
      if (x > ov || (x == ov && e < ok)) { ov = x; ok = e; }
    }
  };
  for (int b = g + wv * G; b < M; b += NW * G)  // the first block, upper triangle
    for (int a = lane; a <= b; a += 64) consider(0, a, b, A[(int64_t)b * M + a]);
  __syncthreads();
  const int nown = (M - g + G - 1) / G, nch = (M + 255) / 256;
  int i = 0, it = 0;
  while (i < M) {
    const int w = M - i;
    argmax2(bv, bk, ov, ok);
    S22Cand* sl = slots + (it & 1) * G;
    if (tid == 0) sl[g] = S22Cand{bv, ov, bk, ok};
    grid.sync();
    bv = -1.0; ov = -1.0; bk = INT_MAX; ok = INT_MAX;
    if (tid < G) { const S22Cand c = sl[tid]; bv = c.dv; bk = c.dk; ov = c.ov; ok = c.ok; }
    argmax2(bv, bk, ov, ok);
    const double gd = bv, go = (w > 1) ? ov : 0.0;
    const int kd = bk, s_r = (w > 1) ? ok / w : 0, s_c = (w > 1) ? ok % w : 0;
    bv = -1.0; ov = -1.0; bk = INT_MAX; ok = INT_MAX;
    int mode;
    if (gd == 0.0 && go == 0.0) mode = 0;
    else if (gd >= alpha * go) mode = 1;
    else mode = 2;
    if (mode == 0) break;
    __syncthreads();  // every thread has read perm / pos of the last step
    if (tid == 0) {
      auto swp = [&](int x, int y) {
        const int32_t u = perm[x], v = perm[y];
        perm[x] = v; perm[y] = u; pos[v] = x; pos[u] = y;
      };
      if (mode == 1) swp(i, i + kd);
      else { swp(i, i + s_r); swp(i + 1, i + s_c); }
    }
    __syncthreads();
    const int p = perm[i], q = mode == 2 ? perm[i + 1] : p;
    const int i0 = i + mode;
    const double* Ap = A + (int64_t)p * M;
    const double* Aq = A + (int64_t)q * M;
    if (mode == 1) {
      const double d = Ap[p];
      for (int a = tid; a < M; a += NT)
        if (pos[a] >= i0) l0[a] = Ap[a] / d;
      if (g == 0 && tid == 0) { at(D, M, i, i) = d; mags[i] = fabs(d); }
    } else {
      const double e11 = Ap[p], e12 = Ap[q], e22 = Aq[q];
      const double det = e11 * e22 - e12 * e12;
      for (int a = tid; a < M; a += NT)
        if (pos[a] >= i0) {
          const double c1 = Ap[a], c2 = Aq[a];
          l0[a] = (c1 * e22 - c2 * e12) / det;
          l1[a] = (c2 * e11 - c1 * e12) / det;
        }
      if (g == 0 && tid == 0) {
        at(D, M, i, i) = e11; at(D, M, i + 1, i) = e12; at(D, M, i, i + 1) = e12; at(D, M, i + 1, i + 1) = e22;
        const double h = 0.5 * (e11 + e22), qq = sqrt(0.25 * (e11 - e22) * (e11 - e22) + e12 * e12);
        const double mg = fmin(fabs(h - qq), fabs(h + qq));
        mags[i] = mg; mags[i + 1] = mg;
        bsize[i] = 2; bsize[i + 1] = 0;
      }
    }
    __syncthreads();
    if (g == 0)
      for (int a = tid; a < M; a += NT)
        if (pos[a] >= i0) {
          Lo[(int64_t)i * M + a] = l0[a];
          if (mode == 2) Lo[(int64_t)(i + 1) * M + a] = l1[a];
        }
    // the 1x1 and 2x2 updates are separate instantiations, each with the
    // expression of the single-workgroup kernel
    auto update = [&](auto two) {
      constexpr bool TWO = decltype(two)::value;
      for (int t = wv; t < nown * nch; t += NW) {
        const int j = t / nch, ch = t - j * nch;
        const int b = g + j * G;
        const int pb = pos[b];
        if (pb < i0) continue;
        double* Ab = A + (int64_t)b * M;
        const double cp = TWO ? Ap[b] : Ab[p];  // A(p, b); A(b, p) and A(b, q) for a 2x2 pivot
        const double cq = TWO ? Aq[b] : 0.0;
        const int a0 = ch * 256 + lane;
        double x[4];
        int pa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = a0 + 64 * u;
          pa[u] = a < M ? pos[a] : -1;
          x[u] = pa[u] >= i0 ? Ab[a] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = a0 + 64 * u;
          if (pa[u] >= i0) {
            double v;
            if constexpr (TWO) v = x[u] - (l0[a] * cp + l1[a] * cq);
            else v = x[u] - l0[a] * cp;
            Ab[a] = v;
            consider(i0, pa[u] - i0, pb - i0, v);
          }
        }
      }
    };
    if (mode == 1) update(std::false_type{});
    else update(std::true_type{});
    __syncthreads();
    i = i0;
    ++it;
  }
  if (g != 0) return;
  for (int e = tid; e < M; e += NT) perm_out[e] = perm[e];
  if (tid == 0) {
    int t = M;
    double prev = 1.0;
    for (int q = 0; q < M; ++q) {
      if (mags[q] == 0.0 || mags[q] < tau * prev) { t = q; break; }
      prev = mags[q];
    }
    const int postponed = M - t;
    const int e = postponed > 0 ? min(n_enlarge, t) : 0;
    int start = t - e;
    if (start > 0 && start < M && bsize[start] == 0) --start;
    int k = 0;
    for (int q = M - 1; q >= start; --q) {
      if (mags[q] <= ker_tol) ++k;
      else break;
    }
    double gap = INFINITY;
    if (k > 0 && start < M - k) {
      double mn = INFINITY, mx = 0.0;
      for (int q = start; q < M - k; ++q) mn = fmin(mn, mags[q]);
      for (int q = M - k; q < M; ++q) mx = fmax(mx, mags[q]);
      gap = mn / fmax(mx, 1e-300);
    }
    info[0] = k;
    info[1] = postponed;
    info[2] = M - start;
    info[3] = gap;
  }
}

// L in position order from Lo (rows by original index): L(r, j) = Lo(perm_r, j)
// below the diagonal, 1 on it, 0 above
__global__ void k_s22_lorder(int M, const double* __restrict__ Lo, const int32_t* __restrict__ perm,
                             double* __restrict__ L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)M * M) return;
  const int j = (int)(e / M), r = (int)(e - (int64_t)j * M);
  L[e] = r == j ? 1.0 : (r > j ? Lo[(int64_t)j * M + perm[r]] : 0.0);
}

// Launches k_s22_ldlt_grid when the device runs cooperative grids that hold one
// workgroup per CU; false (nothing launched) otherwise.
static bool s22_ldlt_grid(hf_ctx* ctx, int M, double* A, double* Lo, double* D, int32_t* perm, int32_t* bs,
                          hipStream_t s) {
  int dev = 0, coop = 0, ncu = 0, nb = 0;
  HF_HIP(hipGetDevice(&dev));
  HF_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  HF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  size_t lds = (size_t)M * (2 * sizeof(double) + 2 * sizeof(int32_t));
  HF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_s22_ldlt_grid, S22_NT, lds));
  if (!coop || nb < 1 || ncu < 1) return false;
  int G = std::min(ncu, (M + 15) / 16);  // about 16 columns per workgroup
  ctx->d_s22slots.alloc((size_t)2 * G * sizeof(S22Cand));
  S22Cand* slots = ctx->d_s22slots.as<S22Cand>();
  double* mags = ctx->d_s22mag.as<double>();
  double* info = ctx->d_s22info.as<double>();
  double tau = ctx->opt.tau, ker_tol = ctx->opt.ker_tol;
  int n_enlarge = ctx->opt.n_enlarge;
  void* args[] = {&M, &A, &Lo, &D, &perm, &mags, &bs, &tau, &n_enlarge, &ker_tol, &info, &slots};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_s22_ldlt_grid), dim3(G),
                                                  dim3(S22_NT), args, (unsigned)lds, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// Null vectors of S22: N2 = P^T [-L11^{-T} L21^T; I_k], stored in column chunks
// of KC columns (chunk c: row-major rows x kc at N2 + c rows KC).  One workgroup
// per kernel column q: y = L11^{-T} l with l = row r+q of L (first r entries),
// by backward substitution taken a column at a time: each final y_t is
// broadcast and its multiple of row t of L (column t of Lt = L^T) leaves the
// earlier positions, last position first.  y sits in LDS (M doubles) when
// M <= S22_LDS_M, else directly in the rows of N2.
__global__ void __launch_bounds__(1024)
k_s22_null(int M, int k, const double* __restrict__ Lt, const int32_t* __restrict__ perm, int rows,
           double* __restrict__ N2c) {
  extern __shared__ double sm[];
  const int q = blockIdx.x, tid = threadIdx.x, NT = blockDim.x;
  const int r = M - k;
  const bool lds = M <= S22_LDS_M;
  const int kc = min(KC, k - (q / KC) * KC), qc = q % KC;
  double* N2 = N2c + (int64_t)(q / KC) * rows * KC;  // this column's chunk, kc columns
  auto Y = [&](int i) -> double& { return lds ? sm[i] : N2[(int64_t)perm[i] * kc + qc]; };
  const double* l = Lt + (int64_t)(r + q) * M;  // row r+q of L
  for (int i = tid; i < r; i += NT) Y(i) = l[i];
  __syncthreads();
  for (int t = r - 1; t > 0; --t) {
    const double yt = Y(t);
    const double* Lr = Lt + (int64_t)t * M;
    for (int i = tid; i < t; i += NT) Y(i) -= Lr[i] * yt;
    __syncthreads();
  }
  for (int i = tid; i < r; i += NT) {
    const double v = Y(i);
    N2[(int64_t)perm[i] * kc + qc] = -v;
  }
  for (int t = tid; t < k; t += NT) N2[(int64_t)perm[r + t] * kc + qc] = (t == q) ? 1.0 : 0.0;
}

// Lt = L^T for a square column-major M x M matrix (32 x 32 tiles through LDS)
__global__ void __launch_bounds__(256) k_transpose_sq(int M, const double* __restrict__ A, double* __restrict__ At) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int r = bx + tx, c = by + j;
    if (r < M && c < M) tile[j][tx] = A[(int64_t)c * M + r];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = by + tx, c = bx + j;
    if (r < M && c < M) At[(int64_t)c * M + r] = tile[tx][j];
  }
}

// x = S22^+ y restricted to the nonsingular pivots (kernel pivots get 0), for
// M > 64.  Y, X: row-major M x nc.  One workgroup per column.  The forward
// substitution walks the columns of L: z_i loses L_it z_t for t = 0, 1, ... in
// turn, the order of row-by-row substitution.  The backward one subtracts the
// multiple of each final position from the earlier ones, last position first
// (the order of k_s22_solve_w), reading the rows of L as columns of Lt = L^T.
// The work column sits in LDS (M doubles) when M <= S22_LDS_M, else at
// work + c M.
__global__ void __launch_bounds__(1024)
k_s22_solve(int M, int k, const double* __restrict__ L, const double* __restrict__ Lt, const double* __restrict__ D,
            const int32_t* __restrict__ perm, const int32_t* __restrict__ bsize, int nc,
            const double* __restrict__ Y, double* __restrict__ X, double* __restrict__ work) {
  extern __shared__ double sm[];
  const int c = blockIdx.x, tid = threadIdx.x, NT = blockDim.x;
  double* z = M <= S22_LDS_M ? sm : work + (int64_t)c * M;
  for (int i = tid; i < M; i += NT) z[i] = Y[(int64_t)perm[i] * nc + c];
  __syncthreads();
  for (int t = 0; t + 1 < M; ++t) {
    const double zt = z[t];
    const double* Lc = L + (int64_t)t * M;
    for (int i = t + 1 + tid; i < M; i += NT) z[i] -= Lc[i] * zt;
    __syncthreads();
  }
  // D: a 2x2 block is solved by the thread of its first position
  const int r = M - k;
  for (int i = tid; i < M; i += NT) {
    if (i >= r) {
      z[i] = 0.0;
    } else if (bsize[i] == 2 && i + 1 < r) {
      const double e11 = at(const_cast<double*>(D), M, i, i), e12 = at(const_cast<double*>(D), M, i + 1, i);
      const double e22 = at(const_cast<double*>(D), M, i + 1, i + 1);
      const double det = e11 * e22 - e12 * e12;
      const double a = z[i], b = z[i + 1];
      z[i] = (a * e22 - b * e12) / det;
      z[i + 1] = (b * e11 - a * e12) / det;
    } else if (!(i > 0 && bsize[i - 1] == 2)) {
      z[i] = z[i] / at(const_cast<double*>(D), M, i, i);
    }
  }
  __syncthreads();
  for (int t = M - 1; t > 0; --t) {
    const double zt = z[t];
    const double* Lr = Lt + (int64_t)t * M;
    for (int i = tid; i < t; i += NT) z[i] -= Lr[i] * zt;
    __syncthreads();
  }
  for (int i = tid; i < M; i += NT) X[(int64_t)perm[i] * nc + c] = z[i];
}

// The same for M <= 64: one workgroup, each wave takes columns in turn and holds
// one column in its lanes (lane i: position i of the LDL^T), L in LDS.  The
// forward substitution subtracts in the same order as row-by-row substitution;
// the backward one broadcasts each final position and subtracts its multiple
// from the earlier ones (last position first).  The 1x1 / 2x2 pivot solves are
// those of k_s22_solve, lane-parallel (the partner value of a 2x2 block comes
// from the neighbouring lane).
__global__ void __launch_bounds__(1024)
k_s22_solve_w(int M, int k, const double* __restrict__ L, const double* __restrict__ D,
              const int32_t* __restrict__ perm, const int32_t* __restrict__ bsize, int nc,
              const double* __restrict__ Y, double* __restrict__ X) {
  __shared__ double Ls[MAXM * MAXM];   // column-major, as in global memory
  __shared__ double Lst[MAXM * MAXM];  // its transpose: lanes read consecutive words
  for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
    const double x = L[e];
    Ls[e] = x;
    Lst[(e % M) * M + e / M] = x;
  }
  __syncthreads();
  const int i = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int r = M - k;
  // this lane's pivot: 1x1, first or second half of a 2x2 block, or a kernel pivot
  int kind = 0;  // 0: kernel / outside, 1: 1x1, 2: first of a 2x2, 3: second of a 2x2
  double e11 = 0.0, e12 = 0.0, e22 = 0.0;
  if (i < r) {
    if (bsize[i] == 2 && i + 1 < r) kind = 2;
    else if (i > 0 && bsize[i - 1] == 2 && i < r) kind = 3;
    else kind = 1;
    const int b0 = kind == 3 ? i - 1 : i;
    e11 = D[(int64_t)b0 * M + b0];
    if (kind >= 2) {
      e12 = D[(int64_t)b0 * M + b0 + 1];
      e22 = D[(int64_t)(b0 + 1) * M + b0 + 1];
    }
  }
  for (int c = threadIdx.x >> 6; c < nc; c += nw) {
    double z = (i < M) ? Y[(int64_t)perm[i] * nc + c] : 0.0;
    for (int t = 0; t < M; ++t) {
      const double zt = lane_bcast(z, t);
      if (i > t && i < M) z -= Ls[(int64_t)t * M + i] * zt;
    }
    // D: 1x1 and 2x2 pivots, kernel pivots set to 0
    const double up = __shfl_down(z, 1, 64), dn = __shfl_up(z, 1, 64);
    if (kind == 1) z = z / e11;
    else if (kind == 2) z = (z * e22 - up * e12) / (e11 * e22 - e12 * e12);
    else if (kind == 3) z = (z * e11 - dn * e12) / (e11 * e22 - e12 * e12);
    else z = 0.0;
    for (int t = M - 1; t >= 0; --t) {
      const double zt = lane_bcast(z, t);
      if (i < t) z -= Lst[(int64_t)t * M + i] * zt;
    }
    if (i < M) X[(int64_t)perm[i] * nc + c] = z;
  }
}

// unpivoted Cholesky G = R^T R of a small SPD matrix (row-major k x k, k <= 64);
// coef = R^{-1}.  One wave: lane c owns column c of R (row j of R is formed
// after row j-1, one lane per entry) and then column c of R^{-1} (back
// substitution); R stays in LDS.
__global__ void __launch_bounds__(64) k_chol_inv(int k, const double* __restrict__ G, double* __restrict__ Rinv) {
  __shared__ double R[MAXM * MAXM];
  const int c = threadIdx.x;
  for (int e = c; e < k * k; e += 64) R[e] = 0.0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double s = G[j * k + j];
    for (int t = 0; t < j; ++t) s -= R[t * k + j] * R[t * k + j];
    s = sqrt(fmax(s, 0.0));
    if (c > j && c < k) {
      double v = G[j * k + c];
      for (int t = 0; t < j; ++t) v -= R[t * k + j] * R[t * k + c];
      R[j * k + c] = s > 0.0 ? v / s : 0.0;
    }
    if (c == j) R[j * k + j] = s;
    __syncthreads();
  }
  if (c >= k) return;
  for (int i = k - 1; i > c; --i) Rinv[i * k + c] = 0.0;
  for (int i = c; i >= 0; --i) {
    double v = (i == c) ? 1.0 : 0.0;
    for (int t = i + 1; t <= c; ++t) v -= R[i * k + t] * Rinv[t * k + c];
    Rinv[i * k + c] = R[i * k + i] > 0.0 ? v / R[i * k + i] : 0.0;
  }
}

// kernel lift in elimination order -> original order, scaled by Q:
// Nout[perm[g], q] = qp[g] * Nin[g, q], with rows of the hard part set from N2.
__global__ void k_kernel_finish(int64_t n, int k, const int32_t* __restrict__ perm,
                                const double* __restrict__ qp, const double* __restrict__ Nin,
                                double* __restrict__ Nout) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = e / k;
  const int q = (int)(e - g * k);
  if (g >= n) return;
  Nout[(int64_t)perm[g] * k + q] = qp[g] * Nin[e];
}

__global__ void k_set_rows(int M, int k, const int32_t* __restrict__ l2, const double* __restrict__ N2,
                           double* __restrict__ N) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * k) return;
  const int i = e / k, q = e - (e / k) * k;
  N[(int64_t)l2[i] * k + q] = N2[e];
}

// user B (col-major, original order) -> b (row-major, elimination order, scaled)
__global__ void k_load_rhs(int64_t n, int m, const int32_t* __restrict__ perm, const double* __restrict__ qp,
                           const double* __restrict__ B, int64_t ldb, int c0, double* __restrict__ b) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = e / m;
  const int c = (int)(e - g * m);
  if (g >= n) return;
  b[e] = qp[g] * B[(int64_t)(c0 + c) * ldb + perm[g]];
}

__global__ void k_mask_rows(int64_t n, int m, const uint8_t* __restrict__ isl2, const double* __restrict__ in,
                            double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = e / m;
  if (g >= n) return;
  out[e] = isl2[g] ? 0.0 : in[e];
}

// x (row-major elimination order) -> xo (row-major original order), scaled
__global__ void k_unperm(int64_t n, int m, const int32_t* __restrict__ perm, const double* __restrict__ qp,
                         const double* __restrict__ x, double* __restrict__ xo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = e / m;
  const int c = (int)(e - g * m);
  if (g >= n) return;
  xo[(int64_t)perm[g] * m + c] = qp[g] * x[e];
}

__global__ void k_store_cols(int64_t n, int m, const double* __restrict__ xo, double* __restrict__ X,
                             int64_t ldx, int c0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = e / m;
  const int c = (int)(e - o * m);
  if (o >= n) return;
  X[(int64_t)(c0 + c) * ldx + o] = xo[e];
}

__global__ void k_neg(int64_t nm, double* __restrict__ a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nm) a[e] = -a[e];
}

__global__ void k_reorder_s22(int M, const int32_t* __restrict__ order, const double* __restrict__ S,
                              double* __restrict__ out, int64_t lds) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int a = e % M, b = e / M;
  out[(int64_t)b * lds + a] = S[(int64_t)order[b] * M + order[a]];
}

__global__ void k_scatter_q(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ qp,
                            double* __restrict__ q) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) q[perm[g]] = qp[g];
}

__global__ void k_kernel_out(int64_t n, int k, const double* __restrict__ N, double* __restrict__ out,
                             int64_t ldn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = e / k;
  const int q = (int)(e - o * k);
  if (o >= n) return;
  const int c = q / KC, kc = min(KC, k - c * KC);
  out[(int64_t)q * ldn + o] = N[(int64_t)c * n * KC + o * kc + (q - c * KC)];
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

struct BgcrWork {
  int64_t n = 0;
  int m = 0, kw = 0, slots = 0;
  DBuf P, Qv, R, Z, T1, partial, gram, Lc, piv, rank, coef, norms;
  // the convergence test's column norms come back through pinned host memory,
  // and the host polls an event for them (a blocking wait wakes up later)
  double* hnorm = nullptr;
  hipEvent_t ready = nullptr;
  ~BgcrWork() {
    if (hnorm) (void)hipHostFree(hnorm);
    if (ready) (void)hipEventDestroy(ready);
  }
};

void free_work(hf_ctx* ctx) {
  delete ctx->work;
  ctx->work = nullptr;
}

// Work space of block GCR on m columns; kw: widest block of the kernel basis a
// Gram product will pair with them (sizes the partial sums only).
static BgcrWork& get_work(hf_ctx* ctx, int m, int kw = 0) {
  if (!ctx->work) {
    auto* nw = new BgcrWork();
    ctx->work = nw;
    HF_HIP(hipHostMalloc((void**)&nw->hnorm, sizeof(double) * MAXM, hipHostMallocDefault));
    HF_HIP(hipEventCreateWithFlags(&nw->ready, hipEventDisableTiming));
  }
  BgcrWork& w = *ctx->work;
  const int slots = ctx->opt.gcr_maxit + 1;
  if (w.n != ctx->n || w.m < m || w.kw < kw || w.slots < slots) {
    const int mm = std::max(m, w.m);
    const int pw = std::max(std::max(mm, kw), w.kw);
    const size_t vec = (size_t)std::max<int64_t>(ctx->n, 1) * mm * sizeof(double);
    w.P.alloc(vec * slots);
    w.Qv.alloc(vec * slots);
    w.R.alloc(vec);
    w.Z.alloc(vec);
    w.T1.alloc(vec);
    w.partial.alloc((size_t)slots * GRAM_WG * pw * pw * sizeof(double));
    w.gram.alloc((size_t)slots * MAXM * MAXM * sizeof(double));
    w.Lc.alloc((size_t)slots * MAXM * MAXM * sizeof(double));
    w.piv.alloc((size_t)slots * MAXM * sizeof(int32_t));
    w.rank.alloc((size_t)slots * sizeof(int32_t));
    w.coef.alloc((size_t)slots * MAXM * MAXM * sizeof(double));
    w.norms.alloc((size_t)MAXM * sizeof(double));
    w.n = ctx->n;
    w.m = mm;
    w.kw = pw;
    w.slots = slots;
  }
  return w;
}

// C (nA blocks of a x b) = [A_blk^T B]
static void gram(hf_ctx* ctx, int64_t n, int a, const double* A, int64_t sA, int nA, int b,
                 const double* B, double* C, hipStream_t s) {
  BgcrWork& w = *ctx->work;
  dim3 grid(GRAM_WG, nA);
  const double by = (double)n * (a * (double)nA + b) * 8.0, fl = 2.0 * n * a * b * (double)nA;
  launch_timed(ctx->timer, HF_K_GRAM, by, fl, s, k_gram_partial, grid, dim3(256), n, a, A, sA, b, B,
               w.partial.as<double>());
  timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, [&] {
    k_gram_reduce<<<cdiv((int64_t)nA * a * b, 64), 1024, 0, s>>>(nA, a * b, w.partial.as<double>(), C);
  });
}

// rows [lo, hi) of Y = K11 W (hi < 0: all rows)
static void spmm_k11(hf_ctx* ctx, int m, const double* W, double* Y, hipStream_t s, int64_t lo = 0,
                     int64_t hi = -1) {
  if (hi < 0) hi = ctx->n;
  const int64_t nr = hi - lo, nm = nr * m;
  if (nm <= 0) return;
  const double frac = ctx->n ? (double)nr / (double)ctx->n : 0.0;
  const double by = frac * ctx->nnz * 12.0 + nr * 8.0 + 2.0 * nm * 8.0, fl = 2.0 * frac * ctx->nnz * m;
  launch_timed(ctx->timer, HF_K_SPMM, by, fl, s, k_spmm_k11, dim3((unsigned)cdiv(nr * ((m + 1) / 2), 256)),
               dim3(256), lo, hi,
               ctx->d_pindptr.as<int64_t>(), ctx->d_pindices.as<int32_t>(), ctx->d_kval.as<double>(),
               ctx->d_isl2.as<uint8_t>(), m, W, Y);
}

// out (n x b) = base + sum_t V_t (n x a) C_t (a x b), row-major blocks
// rng (device, two per term, or nullptr): the rows outside which a term is zero
static void combine(hf_ctx* ctx, int64_t n, int a, int b, double* out, const double* base, int nterms,
                    const double* V, int64_t sV, const double* coef, hipStream_t s,
                    const int64_t* rng = nullptr) {
  if (n * b == 0) return;
  if (a % CKB) rng = nullptr;
  // algorithmic rows of V: all n per term, or (rng, which is only ever the row
  // ranges of X12's blocks) the rows each term covers
  double vrows = (double)nterms * n;
  if (rng) {
    vrows = 0.0;
    for (int t = 0; t < nterms; ++t) vrows += (double)(ctx->x12_rng[2 * t + 1] - ctx->x12_rng[2 * t]);
  }
  const double by = (vrows * a + (base ? 2.0 : 1.0) * n * b) * 8.0;
  const double fl = 2.0 * vrows * a * b;
  launch_timed(ctx->timer, HF_K_COMBINE, by, fl, s, k_combine, dim3((unsigned)cdiv(n, 64)), dim3(256), n, a, b, out,
               base, nterms, V, sV, coef, rng);
}

// row ranges of the blocks of X12 (nullptr for a single tree: every row)
static const int64_t* x12_rows(hf_ctx* ctx) {
  return ctx->n_roots > 1 && ctx->nblk > 0 ? ctx->d_x12rng.as<int64_t>() : nullptr;
}

static void precond(hf_ctx* ctx, int m, const double* R, double* Y, hipStream_t s, int64_t lo = 0,
                    int64_t hi = -1) {
  if (ctx->factor_prec == HF_PREC_FP32) precond_apply<float>(ctx, m, R, Y, s, lo, hi);
  else precond_apply<double>(ctx, m, R, Y, s, lo, hi);
}

// Algorithm 5 on A = K11 for m right-hand sides B (row-major n x m, zero on the
// hard part); X receives the solution.  Returns the iteration count.
static int bgcr(hf_ctx* ctx, int m, const double* B, double* X, double tol, hipStream_t s, int64_t lo = 0,
                int64_t hi = -1) {
  // rows [lo, hi) carry the iteration: outside them B is zero and K11 couples
  // nothing to them (whole trees of a forest), so X is zero there (set after the
  // first preconditioner application) and every other vector is only read and
  // written inside
  if (hi < 0) hi = ctx->n;
  const int64_t n = hi - lo;
  const int64_t nm = n * m;
  BgcrWork& w = get_work(ctx, m);
  const int64_t sv = ctx->n * m;  // slot stride: whole vectors (the preconditioner writes all rows)
  const int64_t o = lo * m;  // offset of the rows that carry the iteration
  double* P = w.P.as<double>() + o;
  double* Qv = w.Qv.as<double>() + o;
  double* R = w.R.as<double>() + o;
  double* Z = w.Z.as<double>() + o;
  const double* Bo = B + o;
  double* Xo = X + o;
  double* G = w.gram.as<double>();
  double* Lc = w.Lc.as<double>();
  int32_t* piv = w.piv.as<int32_t>();
  int32_t* rank = w.rank.as<int32_t>();
  double* coef = w.coef.as<double>();
  const double rel = 1e-14;
  std::vector<double> hb(m * m), hr(m * m);
  std::vector<double> bn2(m);
  // squared column norms, on the host
  double* nrm = w.norms.as<double>();
  auto colsq = [&](const double* Rd, double* out) {
    launch_timed(ctx->timer, HF_K_GRAM, (double)n * m * 8.0, 2.0 * n * m, s, k_colsq_partial, dim3(GRAM_WG),
                 dim3(256), n, m, Rd, w.partial.as<double>());
    launch_timed(ctx->timer, HF_K_OTHER, 0.0, 0.0, s, k_colsq_reduce, dim3(1), dim3(1024), m,
                 (const double*)w.partial.as<double>(), nrm);
    HF_HIP(hipMemcpyAsync(w.hnorm, nrm, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HF_HIP(hipEventRecord(w.ready, s));
    for (;;) {
      const hipError_t e = hipEventQuery(w.ready);
      if (e == hipSuccess) break;
      if (e != hipErrorNotReady) HF_HIP(e);
    }
    std::copy(w.hnorm, w.hnorm + m, out);
  };
  // ||b_k||^2
  colsq(Bo, hb.data());
  for (int k = 0; k < m; ++k) bn2[k] = hb[k];
  // the run's residual history (max relative residual over the active columns)
  struct HistEnd {
    hf_ctx* c;
    ~HistEnd() { c->hist_ptr.push_back((int32_t)c->hist.size()); }
  } hist_end{ctx};
  auto converged = [&](const double* Rd) {
    colsq(Rd, hr.data());
    bool ok = true;
    double worst = 0.0;
    for (int k = 0; k < m; ++k) {
      if (bn2[k] <= 0.0) continue;
      const double rr = hr[k];
      if (!(rr <= tol * tol * bn2[k])) ok = false;
      worst = std::max(worst, std::sqrt(rr / bn2[k]));
    }
    ctx->hist.push_back(worst);
    return ok;
  };
  // X0 = Q^{-1} B, R0 = B - A X0
  precond(ctx, m, B, X, s, lo, hi);
  if (lo > 0 || hi < ctx->n) {  // the preconditioner need not write the rows outside: X is zero there
    if (lo > 0) HF_HIP(hipMemsetAsync(X, 0, (size_t)lo * m * sizeof(double), s));
    if (hi < ctx->n) HF_HIP(hipMemsetAsync(X + hi * m, 0, (size_t)(ctx->n - hi) * m * sizeof(double), s));
  }
  spmm_k11(ctx, m, X, Z - o, s, lo, hi);
  k_sub<<<cdiv(nm, 256), 256, 0, s>>>(nm, Bo, Z, R);
  if (converged(R)) return 0;
  // P0 = Q^{-1} R0, Qv0 = A P0, M0
  precond(ctx, m, R - o, P - o, s, lo, hi);
  spmm_k11(ctx, m, P - o, Qv - o, s, lo, hi);
  gram(ctx, n, m, Qv, 0, 1, m, Qv, G, s);
  k_chol_piv<<<1, 256, 0, s>>>(m, G, 0, Lc, piv, rank, rel);
  const int maxit = ctx->opt.gcr_maxit;
  for (int it = 0; it < maxit; ++it) {
    double* Pn = P + it * sv;
    double* Qn = Qv + it * sv;
    // alpha = M_n^{-1} Qv_n^T R
    gram(ctx, n, m, Qn, 0, 1, m, R, G, s);
    k_chol_solve<<<1, 1024, 0, s>>>(m, m, Lc + (int64_t)it * m * m, piv + (int64_t)it * m, rank + it, G, 0,
                                  coef, 0, 1.0);
    combine(ctx, n, m, m, Xo, Xo, 1, Pn, 0, coef, s);
    k_neg<<<cdiv((int64_t)m * m, 256), 256, 0, s>>>((int64_t)m * m, coef);
    combine(ctx, n, m, m, R, R, 1, Qn, 0, coef, s);
    HF_HIP(hipGetLastError());
    if (converged(R)) return it + 1;
    if (it + 1 >= maxit) break;
    // W = Q^{-1} R -> P_{n+1}; Z = A W -> Qv_{n+1}
    double* Pn1 = P + (it + 1) * sv;
    double* Qn1 = Qv + (it + 1) * sv;
    precond(ctx, m, R - o, Pn1 - o, s, lo, hi);
    spmm_k11(ctx, m, Pn1 - o, Qn1 - o, s, lo, hi);
    // beta_m = -M_m^{-1} Qv_m^T Z, for m = 0..n
    const int nb = it + 1;
    gram(ctx, n, m, Qv, sv, nb, m, Qn1, G, s);
    // the nb coefficient solves at once, one workgroup each
    k_chol_solve<<<nb, 1024, 0, s>>>(m, m, Lc, piv, rank, G, (int64_t)m * m, coef, (int64_t)m * m, -1.0);
    combine(ctx, n, m, m, Pn1, Pn1, nb, P, sv, coef, s);
    combine(ctx, n, m, m, Qn1, Qn1, nb, Qv, sv, coef, s);
    gram(ctx, n, m, Qn1, 0, 1, m, Qn1, G, s);
    k_chol_piv<<<1, 256, 0, s>>>(m, G, 0, Lc + (int64_t)(it + 1) * m * m, piv + (int64_t)(it + 1) * m,
                                rank + it + 1, rel);
    HF_HIP(hipGetLastError());
  }
  throw Status{HF_ERR_NO_CONVERGENCE};
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int factorize_impl(hf_ctx* ctx, const double* values, hipStream_t s) {
  if (ctx->state < 1) return HF_ERR_STATE;
  if (ctx->nnz > 0 && !values) return HF_ERR_ARG;
  const int64_t n = ctx->n;
  try {
    ctx->state = 1;
    auto t0 = std::chrono::steady_clock::now();
    ctx->hist.clear();
    ctx->hist_ptr.assign(1, 0);
    ctx->hist_factor_runs = 0;
    // storage precision of the fronts and factor (FP32 also for FP16 products)
    ctx->factor_prec = ctx->opt.low_precision == HF_PREC_FP64 ? HF_PREC_FP64 : HF_PREC_FP32;
    if (ctx->factor_prec == HF_PREC_FP32) step1<float>(ctx, values, s);
    else step1<double>(ctx, values, s);
    // step 2: the split
    std::vector<uint8_t> isl2(n);
    std::vector<NodeState> hst(ctx->n_nodes);
    if (n) HF_HIP(hipMemcpyAsync(isl2.data(), ctx->d_isl2.ptr, n, hipMemcpyDeviceToHost, s));
    if (ctx->n_nodes)
      HF_HIP(hipMemcpyAsync(hst.data(), ctx->d_state.ptr, sizeof(NodeState) * ctx->n_nodes,
                            hipMemcpyDeviceToHost, s));
    // the sign test of the node inverses (FP32, default mode): which levels the
    // sweeps take in one product
    const bool ninv = !ctx->ninv_copy.empty();
    std::vector<int32_t> bad(ninv ? ctx->n_nodes : 0);
    if (ninv)
      HF_HIP(hipMemcpyAsync(bad.data(), ctx->d_ninv_bad.ptr, sizeof(int32_t) * bad.size(), hipMemcpyDeviceToHost,
                            s));
    HF_HIP(hipStreamSynchronize(s));
    ctx->hstate = hst;
    {
      const int nlev = (int)ctx->level_ptr.size() - 1;
      ctx->level_one_pass.assign(std::max(nlev, 0), 0);
      for (int l = 0; l < nlev; ++l) {
        bool one = ninv && ctx->level_maxp[l] > HF_SWEEP_STEP;
        for (int32_t q = ctx->level_ptr[l]; one && q < ctx->level_ptr[l + 1]; ++q)
          if (bad[ctx->level_nodes[q]]) one = false;
        ctx->level_one_pass[l] = one;
      }
    }
    ctx->lambda2.clear();
    for (int64_t g = 0; g < n; ++g)
      if (isl2[g]) ctx->lambda2.push_back((int32_t)g);
    const int M = (int)ctx->lambda2.size();
    ctx->M = M;
    ctx->flops_done = 0.0;
    for (int32_t j = 0; j < ctx->n_nodes; ++j) {
      const double pt = hst[j].npiv, f = ctx->nodes[j].f;
      ctx->flops_done += pt * f * f - pt * pt * f + pt * pt * pt / 3.0;
    }
    upload(ctx->d_l2, ctx->lambda2, s);
    ctx->t_step1 = ms_since(t0);
    // step 3: K11 X12 = K12 by block GCR, column blocks of width mb
    t0 = std::chrono::steady_clock::now();
    const int mb = ctx->opt.gcr_block > 0 ? std::min(ctx->opt.gcr_block, std::max(M, 1))
                                          : std::min(std::max(M, 1), MAXM);  // 0: all columns (<= 64)
    ctx->mb = mb;
    ctx->nblk = M > 0 ? (M + mb - 1) / mb : 0;
    ctx->gcr_blocks = ctx->nblk;
    ctx->gcr_iters_max = ctx->gcr_iters_total = 0;
    ctx->d_X12.alloc((size_t)std::max(ctx->nblk, 1) * std::max<int64_t>(n, 1) * mb * sizeof(double));
    double* X12 = ctx->d_X12.as<double>();
    ctx->x12_rng.assign((size_t)2 * ctx->nblk, 0);
    if (M > 0) {
      BgcrWork& w = get_work(ctx, mb);
      double* Bk = w.T1.as<double>();
      for (int blk = 0; blk < ctx->nblk; ++blk) {
        const int c0 = blk * mb, nbc = std::min(mb, M - c0);
        HF_HIP(hipMemsetAsync(Bk, 0, (size_t)n * mb * sizeof(double), s));
        k_gather_k12<<<nbc, 256, 0, s>>>(ctx->d_pindptr.as<int64_t>(), ctx->d_pindices.as<int32_t>(),
                                         ctx->d_kval.as<double>(), ctx->d_isl2.as<uint8_t>(),
                                         ctx->d_l2.as<int32_t>(), c0, nbc, mb, Bk);
        // the rows of the trees the block's columns live in (K11 couples no two
        // trees of a forest; a single tree: all rows)
        int64_t lo = n, hi = 0;
        for (int c = c0; c < c0 + nbc; ++c) {
          const int32_t r = ctx->row_tree[ctx->lambda2[c]];
          lo = std::min(lo, ctx->tree_lo[r]);
          hi = std::max(hi, ctx->tree_hi[r]);
        }
        if (ctx->n_roots <= 1 || lo >= hi) lo = 0, hi = n;
        ctx->x12_rng[2 * blk] = lo;
        ctx->x12_rng[2 * blk + 1] = hi;
        const int its = bgcr(ctx, mb, Bk, X12 + (int64_t)blk * n * mb, ctx->opt.gcr_tol, s, lo, hi);
        ctx->gcr_iters_max = std::max(ctx->gcr_iters_max, its);
        ctx->gcr_iters_total += its;
      }
    }
    // the rows each block of X12 lives in, for the products over all of X12
    if (ctx->n_roots > 1 && ctx->nblk > 0) upload(ctx->d_x12rng, ctx->x12_rng, s);
    ctx->hist_factor_runs = (int32_t)ctx->hist_ptr.size() - 1;
    ctx->t_gcr = ms_since(t0);
    // step 4: S22 = K22 - K21 X12 (symmetrized); step 5: its LDL^T and kernel
    t0 = std::chrono::steady_clock::now();
    ctx->d_S22.alloc((size_t)std::max(M, 1) * std::max(M, 1) * sizeof(double));
    ctx->d_S22f.alloc((size_t)std::max(M, 1) * std::max(M, 1) * sizeof(double) * 4);
    ctx->d_s22perm.alloc((size_t)std::max(M, 1) * sizeof(int32_t) * 2);
    if (M > 46340) throw Status{HF_ERR_NOT_IMPLEMENTED};  // S22 positions are int32 in its factorization
    ctx->d_s22mag.alloc((size_t)std::max(M, 1) * sizeof(double));
    ctx->d_s22info.alloc(8 * sizeof(double));
    double* S = ctx->d_S22.as<double>();
    double* Aw = ctx->d_S22f.as<double>();
    double* Lw = Aw + (int64_t)std::max(M, 1) * std::max(M, 1);
    double* Dw = Lw + (int64_t)std::max(M, 1) * std::max(M, 1);
    double* Lo = Dw + (int64_t)std::max(M, 1) * std::max(M, 1);  // L by original row (grid factorization)
    int32_t* sperm = ctx->d_s22perm.as<int32_t>();
    int32_t* sbs = sperm + std::max(M, 1);
    ctx->kdim = 0;
    ctx->rank_gap = INFINITY;
    ctx->rank_candidates = 0;
    if (M > 0) {
      for (int blk = 0; blk < ctx->nblk; ++blk) {
        const int c0 = blk * mb, nbc = std::min(mb, M - c0);
        k_s22_block<<<cdiv((int64_t)M * nbc, 256), 256, 0, s>>>(
            ctx->d_pindptr.as<int64_t>(), ctx->d_pindices.as<int32_t>(), ctx->d_kval.as<double>(),
            ctx->d_isl2.as<uint8_t>(), ctx->d_l2.as<int32_t>(), M, c0, nbc, mb, X12 + (int64_t)blk * n * mb, S);
      }
      k_symmetrize<<<cdiv((int64_t)M * M, 256), 256, 0, s>>>(M, S);
      HF_HIP(hipMemcpyAsync(Aw, S, sizeof(double) * M * M, hipMemcpyDeviceToDevice, s));
      if (M > MAXM && M <= S22_GRID_MAXM && s22_ldlt_grid(ctx, M, Aw, Lo, Dw, sperm, sbs, s))
        k_s22_lorder<<<cdiv((int64_t)M * M, 256), 256, 0, s>>>(M, Lo, sperm, Lw);
      else
        k_s22_ldlt<<<1, S22_NT, 0, s>>>(M, Aw, Lw, Dw, sperm, ctx->d_s22mag.as<double>(), sbs, ctx->opt.tau,
                                     ctx->opt.n_enlarge, ctx->opt.ker_tol, ctx->d_s22info.as<double>());
      // the working copy is spent: it takes L^T, whose columns are the rows of L
      // that the backward substitutions read
      k_transpose_sq<<<dim3(cdiv(M, 32), cdiv(M, 32)), 256, 0, s>>>(M, Lw, Aw);
      double info[4];
      HF_HIP(hipMemcpyAsync(info, ctx->d_s22info.ptr, sizeof(info), hipMemcpyDeviceToHost, s));
      HF_HIP(hipStreamSynchronize(s));
      ctx->kdim = (int)info[0];
      ctx->rank_candidates = (int)info[2];
      ctx->rank_gap = info[3];
    }
    const int k = ctx->kdim;
    if (k > KMAX) throw Status{HF_ERR_NOT_IMPLEMENTED};
    if (k > 0) {
      // lift: N = [-X12 N2; N2], then Q Pi^T, then orthonormalize; KC columns at
      // a time (block Gram-Schmidt against the earlier chunks, CholeskyQR of the
      // chunk, both twice)
      BgcrWork& w = get_work(ctx, mb, std::min(k, KC));
      const int rows = ctx->nblk * mb;
      const int nkc = (k + KC - 1) / KC;
      ctx->d_N2.alloc((size_t)rows * KC * nkc * sizeof(double));
      double* N2 = ctx->d_N2.as<double>();
      HF_HIP(hipMemsetAsync(N2, 0, (size_t)rows * KC * nkc * sizeof(double), s));
      k_s22_null<<<k, 1024, M <= S22_LDS_M ? (size_t)M * sizeof(double) : 0, s>>>(M, k, Aw, sperm, rows, N2);
      ctx->d_kern.alloc((size_t)n * KC * nkc * sizeof(double));
      double* Nall = ctx->d_kern.as<double>();
      ctx->d_ktmp.alloc((size_t)n * KC * 2 * sizeof(double));
      double* Nperm = ctx->d_ktmp.as<double>();
      double* tmp = Nperm + (int64_t)n * KC;
      double* G = w.gram.as<double>();
      double* Ri = w.coef.as<double>();
      for (int c = 0; c < nkc; ++c) {
        const int kc = kchunk(k, c);
        const double* N2c = N2 + (int64_t)c * rows * KC;
        double* Nc = Nall + (int64_t)c * n * KC;
        combine(ctx, n, mb, kc, Nperm, nullptr, ctx->nblk, X12, (int64_t)n * mb, N2c, s, x12_rows(ctx));
        k_neg<<<cdiv(n * kc, 256), 256, 0, s>>>(n * kc, Nperm);
        k_set_rows<<<cdiv((int64_t)M * kc, 256), 256, 0, s>>>(M, kc, ctx->d_l2.as<int32_t>(), N2c, Nperm);
        k_kernel_finish<<<cdiv(n * kc, 256), 256, 0, s>>>(n, kc, ctx->d_perm.as<int32_t>(), ctx->d_q.as<double>(),
                                                          Nperm, Nc);
        for (int pass = 0; pass < 2; ++pass) {
          for (int d = 0; d < c; ++d) {  // Nc -= Nd (Nd^T Nc)
            const double* Nd = Nall + (int64_t)d * n * KC;
            gram(ctx, n, KC, Nd, 0, 1, kc, Nc, G, s);
            k_neg<<<cdiv((int64_t)KC * kc, 256), 256, 0, s>>>((int64_t)KC * kc, G);
            combine(ctx, n, KC, kc, Nc, Nc, 1, Nd, 0, G, s);
          }
          gram(ctx, n, kc, Nc, 0, 1, kc, Nc, G, s);
          k_chol_inv<<<1, 64, 0, s>>>(kc, G, Ri);
          combine(ctx, n, kc, kc, tmp, nullptr, 1, Nc, 0, Ri, s);
          HF_HIP(hipMemcpyAsync(Nc, tmp, (size_t)n * kc * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
      }
    }
    HF_HIP(hipGetLastError());
    HF_HIP(hipStreamSynchronize(s));
    ctx->timer.flush();
    ctx->t_s22 = ms_since(t0);
    ctx->state = 2;
  } catch (const HipError&) {
    return HF_ERR_HIP;
  } catch (const Status& st) {
    return st.code;
  } catch (const std::bad_alloc&) {
    return HF_ERR_OOM;
  }
  return HF_OK;
}

// Algorithm 2 on scaled right-hand sides b (row-major n x m, elimination order):
// x receives [x1; x2].  Scratch: b1 and the block-GCR work space.
static int solve_core(hf_ctx* ctx, int m, const double* b, double* x, double* b1, double tol, hipStream_t s) {
  const int64_t n = ctx->n;
  const int64_t nm = n * m;
  const int M = ctx->M, k = ctx->kdim;
  k_mask_rows<<<cdiv(nm, 256), 256, 0, s>>>(n, m, ctx->d_isl2.as<uint8_t>(), b, b1);
  const int its = bgcr(ctx, m, b1, x, tol, s);  // y1
  if (M > 0) {
    ctx->d_y2.alloc((size_t)M * m * sizeof(double) * 3);
    double* y2 = ctx->d_y2.as<double>();
    double* x2 = y2 + (int64_t)M * m;
    double* wk = x2 + (int64_t)M * m;
    k_y2<<<cdiv((int64_t)M * m, 256), 256, 0, s>>>(ctx->d_pindptr.as<int64_t>(), ctx->d_pindices.as<int32_t>(),
                                                   ctx->d_kval.as<double>(), ctx->d_isl2.as<uint8_t>(),
                                                   ctx->d_l2.as<int32_t>(), M, m, b, x, y2);
    double* S = ctx->d_S22f.as<double>();
    const int64_t MM = (int64_t)M * M;
    int32_t* sperm = ctx->d_s22perm.as<int32_t>();
    if (M <= MAXM)
      k_s22_solve_w<<<1, 1024, 0, s>>>(M, k, S + MM, S + 2 * MM, sperm, sperm + M, m, y2, x2);
    else  // S holds [L^T | L | D]
      k_s22_solve<<<m, 1024, M <= S22_LDS_M ? (size_t)M * sizeof(double) : 0, s>>>(
          M, k, S + MM, S, S + 2 * MM, sperm, sperm + M, m, y2, x2, wk);
    // x1 = y1 - X12 x2 (x2 rows padded per block)
    const int mb = ctx->mb;
    ctx->d_x2pad.alloc((size_t)ctx->nblk * mb * m * sizeof(double));
    double* x2p = ctx->d_x2pad.as<double>();
    HF_HIP(hipMemsetAsync(x2p, 0, (size_t)ctx->nblk * mb * m * sizeof(double), s));
    HF_HIP(hipMemcpyAsync(x2p, x2, (size_t)M * m * sizeof(double), hipMemcpyDeviceToDevice, s));
    k_neg<<<cdiv((int64_t)ctx->nblk * mb * m, 256), 256, 0, s>>>((int64_t)ctx->nblk * mb * m, x2p);
    combine(ctx, n, mb, m, x, x, ctx->nblk, ctx->d_X12.as<double>(), (int64_t)n * mb, x2p, s, x12_rows(ctx));
    k_set_rows<<<cdiv((int64_t)M * m, 256), 256, 0, s>>>(M, m, ctx->d_l2.as<int32_t>(), x2, x);
  }
  HF_HIP(hipGetLastError());
  return its;
}

int solve_impl(hf_ctx* ctx, int32_t r, const double* B, int64_t ldb, double* X, int64_t ldx,
               hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int64_t n = ctx->n;
  if (r < 0 || (r > 0 && n > 0 && (!B || !X || ldb < n || ldx < n))) return HF_ERR_ARG;
  if (r == 0 || n == 0) return HF_OK;
  try {
    auto t0 = std::chrono::steady_clock::now();
    const int k = ctx->kdim;
    ctx->solve_iters = 0;
    ctx->hist_ptr.resize(ctx->hist_factor_runs + 1);
    ctx->hist.resize(ctx->hist_ptr.back());
    for (int c0 = 0; c0 < r; c0 += MAXM) {
      const int m = std::min(MAXM, r - c0);
      BgcrWork& w = get_work(ctx, std::max(m, ctx->mb), std::min(k, KC));
      const int64_t nm = n * m;
      ctx->d_rhs_b.alloc((size_t)nm * sizeof(double) * 6);
      double* b = ctx->d_rhs_b.as<double>();
      double* b1 = b + nm;
      double* x = b1 + nm;
      double* res = x + nm;
      double* xo = res + nm;
      double* dxo = xo + nm;
      // x -> caller's variables, projected orthogonally to the detected kernel
      auto to_orig = [&](const double* xp, double* out) {
        k_unperm<<<cdiv(nm, 256), 256, 0, s>>>(n, m, ctx->d_perm.as<int32_t>(), ctx->d_q.as<double>(), xp, out);
        double* G = w.gram.as<double>();
        for (int c = 0; c * KC < k; ++c) {  // the chunks are orthonormal to each other
          const int kc = kchunk(k, c);
          const double* Nc = ctx->d_kern.as<double>() + (int64_t)c * n * KC;
          gram(ctx, n, kc, Nc, 0, 1, m, out, G, s);
          k_neg<<<cdiv((int64_t)kc * m, 256), 256, 0, s>>>((int64_t)kc * m, G);
          combine(ctx, n, kc, m, out, out, 1, Nc, 0, G, s);
        }
      };
      k_load_rhs<<<cdiv(nm, 256), 256, 0, s>>>(n, m, ctx->d_perm.as<int32_t>(), ctx->d_q.as<double>(), B, ldb,
                                               c0, b);
      ctx->solve_iters = std::max(ctx->solve_iters, solve_core(ctx, m, b, x, b1, ctx->opt.gcr_tol, s));
      to_orig(x, xo);
      // residual correction: xo += P(Q Pi^T Algorithm2(Pi Q (bbar - Kbar xo))); the
      // residual is taken in the caller's variables on the projected iterate (the
      // scaled matrix has an exactly unit diagonal and differs from Q Kbar Q by
      // rounding; Kbar 1 vanishes only up to rounding)
      for (int it = 0; it < ctx->opt.refine_steps; ++it) {
        k_residual_orig<<<cdiv(nm, 256), 256, 0, s>>>(n, ctx->d_pindptr.as<int64_t>(),
                                                      ctx->d_pindices.as<int32_t>(), ctx->d_kbar.as<double>(),
                                                      ctx->d_q.as<double>(), ctx->d_perm.as<int32_t>(), m, B, ldb, c0,
                                                      xo, res);
        ctx->solve_iters =
            std::max(ctx->solve_iters, solve_core(ctx, m, res, x, b1, ctx->opt.refine_tol, s));
        to_orig(x, dxo);
        k_add<<<cdiv(nm, 256), 256, 0, s>>>(nm, xo, dxo);
      }
      k_store_cols<<<cdiv(nm, 256), 256, 0, s>>>(n, m, xo, X, ldx, c0);
      HF_HIP(hipGetLastError());
    }
    HF_HIP(hipStreamSynchronize(s));
    ctx->timer.flush();
    ctx->t_solve = ms_since(t0);
  } catch (const HipError&) {
    return HF_ERR_HIP;
  } catch (const Status& st) {
    return st.code;
  } catch (const std::bad_alloc&) {
    return HF_ERR_OOM;
  }
  return HF_OK;
}

// Q^{-1} of Sec. 3.2 applied to r <= 64 columns in the scaled, permuted
// variables (row-major n x r, elimination order); the hard part's rows of R are
// not read and those of Y are zero.
int precond_impl(hf_ctx* ctx, int32_t r, const double* R, double* Y, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int64_t n = ctx->n;
  if (r < 0 || r > MAXM || (r > 0 && n > 0 && (!R || !Y || R == Y))) return HF_ERR_ARG;
  if (r == 0 || n == 0) return HF_OK;
  try {
    precond(ctx, r, R, Y, s);
    HF_HIP(hipStreamSynchronize(s));
    ctx->timer.flush();
  } catch (const HipError&) {
    return HF_ERR_HIP;
  } catch (const Status& st) {
    return st.code;
  } catch (const std::bad_alloc&) {
    return HF_ERR_OOM;
  }
  return HF_OK;
}

__global__ void k_tune_fill(int64_t ne, double* __restrict__ R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) R[e] = 1.0 + 0.01 * (double)(e % 13);
}

// The sweeps' launch-shape options timed on the current factors; the fastest
// combination stays in the context.
int tune_impl(hf_ctx* ctx, int32_t r, int32_t* front_min, int32_t* wide_min, double* ms, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int64_t n = ctx->n;
  if (r < 1 || r > MAXM) return HF_ERR_ARG;
  const bool fp32 = ctx->factor_prec == HF_PREC_FP32;
  std::vector<int32_t> fms = fp32 ? std::vector<int32_t>{0, 128, 256, 512}
                                  : std::vector<int32_t>{ctx->opt.sweep_front_min};
  std::vector<int32_t> wms = r > 16 ? std::vector<int32_t>{128, 256, 512, 1024}
                                    : std::vector<int32_t>{ctx->opt.sweep_wide_min};
  double best = INFINITY;
  int32_t bf = ctx->opt.sweep_front_min, bw = ctx->opt.sweep_wide_min;
  hipEvent_t ea = nullptr, eb = nullptr;
  const bool timing = ctx->timer.on;
  ctx->timer.on = false;  // the candidates' launches stay out of the per-class counters
  try {
    if (n > 0) {
      ctx->d_tune.alloc((size_t)n * r * 2 * sizeof(double));
      double* R = ctx->d_tune.as<double>();
      double* Y = R + n * r;
      k_tune_fill<<<cdiv(n * r, 256), 256, 0, s>>>(n * r, R);
      HF_HIP(hipEventCreate(&ea));
      HF_HIP(hipEventCreate(&eb));
      for (int32_t fm : fms)
        for (int32_t wm : wms) {
          ctx->opt.sweep_front_min = fm;
          ctx->opt.sweep_wide_min = wm;
          precond(ctx, r, R, Y, s);  // untimed: allocations, caches
          HF_HIP(hipEventRecord(ea, s));
          constexpr int REPS = 3;
          for (int q = 0; q < REPS; ++q) precond(ctx, r, R, Y, s);
          HF_HIP(hipEventRecord(eb, s));
          HF_HIP(hipEventSynchronize(eb));
          float t = 0.f;
          HF_HIP(hipEventElapsedTime(&t, ea, eb));
          if (t / REPS < best) {
            best = t / REPS;
            bf = fm;
            bw = wm;
          }
        }
    }
  } catch (const HipError&) {
    ctx->timer.on = timing;
    return HF_ERR_HIP;
  } catch (const Status& st) {
    ctx->timer.on = timing;
    return st.code;
  } catch (const std::bad_alloc&) {
    ctx->timer.on = timing;
    return HF_ERR_OOM;
  }
  if (ea) (void)hipEventDestroy(ea);
  if (eb) (void)hipEventDestroy(eb);
  ctx->timer.on = timing;
  ctx->opt.sweep_front_min = bf;
  ctx->opt.sweep_wide_min = bw;
  if (front_min) *front_min = bf;
  if (wide_min) *wide_min = bw;
  if (ms) *ms = std::isfinite(best) ? best : 0.0;
  return HF_OK;
}

// Adjoint of the solve.  Not a step of the paper's method: the derivative of the
// solution map of Algorithm 2, taken with one more solve on the same factors.
// For Kbar x = b with ker Kbar fixed and b in its range, x = Kbar^+ b changes by
// dx = -Kbar^+ dKbar x when Kbar moves along perturbations that keep the kernel.
// A loss with gradient g = dl/dx therefore has dl/db = lambda and
// dl/dKbar_ij = -lambda_i x_j, with lambda = Kbar^+ (g projected onto the range).

// caller columns c0 .. c0+m-1 (column-major, original order) -> row-major n x m
__global__ void k_take_cols(int64_t n, int m, const double* __restrict__ G, int64_t ldg, int c0,
                            double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = e / m;
  const int c = (int)(e - o * m);
  if (o >= n) return;
  out[e] = G[(int64_t)(c0 + c) * ldg + o];
}

// value gradient on the caller's pattern: entry e, in row i and column j of the
// caller's CSR arrays, receives -sum_c Lam[i, c] x[j, c], summed over c in
// ascending order.  One thread per entry in the caller's order: the output is
// written contiguously and neighbouring entries read neighbouring rows of the
// column-major X and Lambda.  Workgroups are dispatched to the eight XCDs in
// turn; the grid (a multiple of 8) is remapped so that each XCD takes one
// contiguous eighth of the entries, and rows that share columns of X (grid
// neighbours one plane apart) meet in the same L2.
__global__ void k_value_grad(int64_t nnz, const int32_t* __restrict__ orow, const int32_t* __restrict__ ocol, int r,
                             const double* __restrict__ X, int64_t ldx, const double* __restrict__ Lam, int64_t ldl,
                             double* __restrict__ GV) {
  const int64_t per = gridDim.x / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t e = lb * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int64_t i = orow[e], j = ocol[e];
  double acc = 0.0;
  int c = 0;
  for (; c + 8 <= r; c += 8) {
    double a[8], x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = Lam[(int64_t)(c + u) * ldl + i];
      x[u] = X[(int64_t)(c + u) * ldx + j];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(a[u], x[u], acc);
  }
  for (; c < r; ++c) acc = fma(Lam[(int64_t)c * ldl + i], X[(int64_t)c * ldx + j], acc);
  GV[e] = -acc;
}

int adjoint_impl(hf_ctx* ctx, int32_t r, const double* X, int64_t ldx, const double* G, int64_t ldg,
                 double* Lam, int64_t ldl, double* GV, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int64_t n = ctx->n;
  if (r < 0 || (r > 0 && n > 0 && (!X || !G || !Lam || ldx < n || ldg < n || ldl < n))) return HF_ERR_ARG;
  if (n == 0) return HF_OK;
  try {
    if (r == 0) {
      if (GV) HF_HIP(hipMemsetAsync(GV, 0, (size_t)ctx->nnz * sizeof(double), s));
      HF_HIP(hipStreamSynchronize(s));
      return HF_OK;
    }
    const int k = ctx->kdim;
    const double* Nk = ctx->d_kern.as<double>();
    // right-hand sides g projected onto the range of Kbar (orthogonal to the kernel)
    ctx->d_adj.alloc((size_t)n * r * sizeof(double));
    double* P = ctx->d_adj.as<double>();
    for (int c0 = 0; c0 < r; c0 += MAXM) {
      const int m = std::min(MAXM, r - c0);
      BgcrWork& w = get_work(ctx, std::max(m, ctx->mb), std::min(k, KC));
      const int64_t nm = n * m;
      ctx->d_rhs_b.alloc((size_t)nm * sizeof(double) * 6);
      double* t = ctx->d_rhs_b.as<double>();
      k_take_cols<<<cdiv(nm, 256), 256, 0, s>>>(n, m, G, ldg, c0, t);
      double* C = w.gram.as<double>();
      for (int c = 0; c * KC < k; ++c) {
        const int kc = kchunk(k, c);
        const double* Nc = Nk + (int64_t)c * n * KC;
        gram(ctx, n, kc, Nc, 0, 1, m, t, C, s);
        k_neg<<<cdiv((int64_t)kc * m, 256), 256, 0, s>>>((int64_t)kc * m, C);
        combine(ctx, n, kc, m, t, t, 1, Nc, 0, C, s);
      }
      k_store_cols<<<cdiv(nm, 256), 256, 0, s>>>(n, m, t, P, n, c0);
      HF_HIP(hipGetLastError());
    }
    const int st = solve_impl(ctx, r, P, n, Lam, ldl, s);
    if (st != HF_OK) return st;
    if (GV && ctx->nnz > 0) {
      if (!ctx->d_orow.ptr) {
        // the caller's pattern as (row, column) pairs, once per context
        std::vector<int32_t> orow(ctx->nnz);
        for (int64_t i = 0; i < n; ++i)
          for (int64_t e = ctx->indptr[i]; e < ctx->indptr[i + 1]; ++e) orow[e] = (int32_t)i;
        upload(ctx->d_orow, orow, s);
        upload(ctx->d_ocol, ctx->indices, s);
        HF_HIP(hipStreamSynchronize(s));
      }
      // algorithmic bytes: the (row, column) pairs, the output, X and Lambda once
      const double by = (double)ctx->nnz * (4.0 + 4.0 + 8.0) + 2.0 * n * r * 8.0;
      launch_timed(ctx->timer, HF_K_VALUE_GRAD, by, 2.0 * ctx->nnz * r, s, k_value_grad,
                   dim3((unsigned)(8 * cdiv(cdiv(ctx->nnz, 256), 8))), dim3(256), ctx->nnz, ctx->d_orow.as<int32_t>(),
                   ctx->d_ocol.as<int32_t>(), r, X, ldx, (const double*)Lam, ldl, GV);
      HF_HIP(hipGetLastError());
    }
    HF_HIP(hipStreamSynchronize(s));
    ctx->timer.flush();
  } catch (const HipError&) {
    return HF_ERR_HIP;
  } catch (const Status& st) {
    return st.code;
  } catch (const std::bad_alloc&) {
    return HF_ERR_OOM;
  }
  return HF_OK;
}

// accessors used by the C entry points
int schur_impl(const hf_ctx* ctx, int32_t* m, int32_t* lambda2, double* S, int64_t lds, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int M = ctx->M;
  *m = M;
  if (!lambda2 && !S) return HF_OK;
  std::vector<std::pair<int32_t, int32_t>> ord(M);
  for (int i = 0; i < M; ++i) ord[i] = {ctx->perm[ctx->lambda2[i]], i};
  std::sort(ord.begin(), ord.end());
  if (lambda2)
    for (int i = 0; i < M; ++i) lambda2[i] = ord[i].first;
  if (S && M > 0) {
    if (lds < M) return HF_ERR_ARG;
    try {
      std::vector<int32_t> order(M);
      for (int i = 0; i < M; ++i) order[i] = ord[i].second;
      DBuf d_order;
      upload(d_order, order, s);
      k_reorder_s22<<<cdiv((int64_t)M * M, 256), 256, 0, s>>>(M, d_order.as<int32_t>(), ctx->d_S22.as<double>(), S,
                                                             lds);
      HF_HIP(hipGetLastError());
      HF_HIP(hipStreamSynchronize(s));
    } catch (const HipError&) {
      return HF_ERR_HIP;
    } catch (const Status& st) {
      return st.code;
    }
  }
  return HF_OK;
}

int kernel_basis_impl(const hf_ctx* ctx, double* N, int64_t ldn, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  const int k = ctx->kdim;
  if (k == 0) return HF_OK;
  if (!N || ldn < ctx->n) return HF_ERR_ARG;
  k_kernel_out<<<cdiv(ctx->n * k, 256), 256, 0, s>>>(ctx->n, k, ctx->d_kern.as<double>(), N, ldn);
  if (hipGetLastError() != hipSuccess) return HF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return HF_ERR_HIP;
  return HF_OK;
}

int scaling_impl(const hf_ctx* ctx, double* q, hipStream_t s) {
  if (ctx->state < 2) return HF_ERR_STATE;
  if (!q) return HF_ERR_ARG;
  if (ctx->n == 0) return HF_OK;
  k_scatter_q<<<cdiv(ctx->n, 256), 256, 0, s>>>(ctx->n, ctx->d_perm.as<int32_t>(), ctx->d_q.as<double>(), q);
  if (hipGetLastError() != hipSuccess) return HF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return HF_ERR_HIP;
  return HF_OK;
}

}  // namespace hf
