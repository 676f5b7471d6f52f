// Step 1 of Algorithm 1 on the GPU: the low-precision multifrontal LDL^T with
// symmetric pivoting on the diagonal and threshold postponing (Sec. 2.1-2.2).
//
// Layout: every tree node j owns a dense column-major front of order
// f_j = p_j + b_j in one HBM arena (T = float or double); rows/columns
// 0..p_j-1 are the node's own indices (pivot candidates), p_j..f_j-1 its border
// (ancestor indices, ascending).  Only the lower triangle is used.  The front is
// factorized in place:
//   F11 (p x p) : blocked right-looking LDL^T.  A panel kernel (one workgroup
//                 per front) picks each pivot by a workgroup argmax over the
//                 eagerly updated diagonal (ties: smallest nested-dissection
//                 index), applies the ratio test of Sec. 2.2, exchanges rows and
//                 columns symmetrically (this also permutes the columns of F21)
//                 and computes the pivot column left-looking within the panel;
//                 a tiled kernel then applies the panel to the trailing F11.
//   F21 (b x p~): L21 = F21 L11^{-T} D^{-1}  (row-strip blocked TRSM)
//   F22 (b x b) : F22 -= L21 D L21^T         (the Schur complement passed to the
//                 parent; rows of postponed indices are not part of it)
// Nodes are processed by height levels: all fronts of a level in the same
// launches, each level after the levels it depends on.
#include <algorithm>
#include <climits>

#include "hf_internal.h"
#include "hf_kernels.h"

namespace hf {

// ---------------------------------------------------------------------------
// F0: scaling of Sec. 2 fused with the assembly of the entries into the fronts
// ---------------------------------------------------------------------------

__global__ void k_scale_q(int64_t n, const int64_t* __restrict__ pindptr,
                          const int32_t* __restrict__ diagpos, const int64_t* __restrict__ psrc,
                          const double* __restrict__ v, double* __restrict__ qp, int* flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double d = v[psrc[pindptr[g] + diagpos[g]]];
  if (!isfinite(d)) atomicOr(flag, 1);
  qp[g] = d != 0.0 ? 1.0 / sqrt(fabs(d)) : 1.0;
}

template <class T>
__global__ void k_scale_assemble(int64_t n, const int64_t* __restrict__ pindptr,
                                 const int32_t* __restrict__ pindices,
                                 const int64_t* __restrict__ psrc, const int64_t* __restrict__ asmmap,
                                 const double* __restrict__ v, const double* __restrict__ qp,
                                 double* __restrict__ kval, double* __restrict__ kbar, T* __restrict__ front,
                                 int* flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double qg = qp[g];
  bool bad = false;
  for (int64_t e = pindptr[g]; e < pindptr[g + 1]; ++e) {
    const double val = v[psrc[e]];
    kbar[e] = val;
    if (!isfinite(val)) bad = true;
    const int32_t c = pindices[e];
    double k;
    if (c == g) k = val > 0.0 ? 1.0 : (val < 0.0 ? -1.0 : 0.0);
    else k = qg * val * qp[c];
    kval[e] = k;
    const int64_t a = asmmap[e];
    if (a >= 0) front[a] = (T)k;
  }
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// F1: extend-add of children's contribution blocks (one launch per child rank,
// so no two writers share a parent element)
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_extend_add(const int32_t* __restrict__ items, int nitems,
                             const NodeInfo* __restrict__ nodes, const int32_t* __restrict__ relmap,
                             T* __restrict__ front) {
  const int it = blockIdx.y;
  if (it >= nitems) return;
  const NodeInfo ci = nodes[items[it]];
  const NodeInfo pi = nodes[ci.parent];
  const int bc = ci.b;
  const int t = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (t >= bc) return;
  const T* C = front + ci.front_off;
  T* F = front + pi.front_off;
  const int32_t* rel = relmap + ci.border_off;
  const int64_t fc = ci.f, fp = pi.f;
  const int64_t ct = (int64_t)(ci.p + t) * fc + ci.p;
  const int64_t pt = (int64_t)rel[t] * fp;
  for (int r = t + (threadIdx.x & 15); r < bc; r += 16) F[pt + rel[r]] += C[ct + r];
}

// ---------------------------------------------------------------------------
// F2: panel factorization of F11 with pivot search and postponing
// ---------------------------------------------------------------------------

template <class T>
__device__ inline void argmax_combine(T& bv, int& bid, int& bk, T v, int id, int k) {
  if (v > bv || (v == bv && id < bid)) { bv = v; bid = id; bk = k; }
}

constexpr int PT = 512;               // threads of the panel kernel
constexpr int PROWS = 4096 / PT;      // rows per thread (nodes hold at most 4096 indices)

template <class T>
__global__ void __launch_bounds__(PT)
k_panel(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes, NodeState* st,
        T* __restrict__ front, int32_t* __restrict__ piv, int32_t* __restrict__ swaps,
        T* __restrict__ dval, int k0p, double tau, int first_unit) {
  const int j = lnodes[blockIdx.x];
  const NodeInfo ni = nodes[j];
  const NodeState s0 = st[j];
  if (s0.done || k0p >= ni.p) return;
  const int p = ni.p;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  int32_t* idx = piv + ni.start;
  int32_t* sw = swaps + ni.start;
  T* D = dval + ni.start;
  const int tid = threadIdx.x;
  constexpr int NW = PT / 64;

  extern __shared__ unsigned char smem_raw[];
  T* dg = reinterpret_cast<T*>(smem_raw);  // current diagonal of positions [k0p, p)
  __shared__ T u[PANEL_NB];
  __shared__ T red_v[NW];
  __shared__ int red_id[NW], red_k[NW];
  __shared__ int s_k, s_stop;

  for (int k = k0p + tid; k < p; k += PT) dg[k - k0p] = F[(int64_t)k * f + k];
  double dprev = s0.dprev;
  int have_prev = (s0.npiv > 0) ? 1 : first_unit;
  const int iend = min(k0p + PANEL_NB, p);
  __syncthreads();
  int i;
  for (i = k0p; i < iend; ++i) {
    // workgroup argmax of |diag| over the remaining candidates
    T bv = (T)-1;
    int bid = INT_MAX, bk = -1;
    for (int k = i + tid; k < p; k += PT) {
      const T v = dg[k - k0p];
      argmax_combine(bv, bid, bk, v < (T)0 ? -v : v, idx[k], k);
    }
    for (int off = 32; off > 0; off >>= 1) {
      const T ov = __shfl_xor(bv, off, 64);
      const int oid = __shfl_xor(bid, off, 64);
      const int ok = __shfl_xor(bk, off, 64);
      argmax_combine(bv, bid, bk, ov, oid, ok);
    }
    if ((tid & 63) == 0) { red_v[tid >> 6] = bv; red_id[tid >> 6] = bid; red_k[tid >> 6] = bk; }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < NW; ++w) argmax_combine(bv, bid, bk, red_v[w], red_id[w], red_k[w]);
      const double dk = (double)dg[bk - k0p];
      int stop = (dk == 0.0);
      if (!stop && have_prev && fabs(dk) < tau * fabs(dprev)) stop = 1;
      s_stop = stop;
      s_k = bk;
      if (!stop) sw[i] = bk;
    }
    __syncthreads();
    if (s_stop) break;
    const int k = s_k;
    if (k != i) {
      // symmetric exchange of positions i < k in the lower triangle; columns of
      // earlier panels get their row exchanges later in one pass (k_apply_swaps)
      for (int c = k0p + tid; c < i; c += PT) {
        const T a = F[(int64_t)c * f + i];
        F[(int64_t)c * f + i] = F[(int64_t)c * f + k];
        F[(int64_t)c * f + k] = a;
      }
      for (int c = i + 1 + tid; c < k; c += PT) {
        const T a = F[(int64_t)i * f + c];
        F[(int64_t)i * f + c] = F[(int64_t)c * f + k];
        F[(int64_t)c * f + k] = a;
      }
      for (int64_t r = k + 1 + tid; r < f; r += PT) {
        const T a = F[(int64_t)i * f + r];
        F[(int64_t)i * f + r] = F[(int64_t)k * f + r];
        F[(int64_t)k * f + r] = a;
      }
      if (tid == 0) {
        const T a = F[(int64_t)i * f + i];
        F[(int64_t)i * f + i] = F[(int64_t)k * f + k];
        F[(int64_t)k * f + k] = a;
        const T dd = dg[i - k0p]; dg[i - k0p] = dg[k - k0p]; dg[k - k0p] = dd;
        const int32_t t = idx[i]; idx[i] = idx[k]; idx[k] = t;
      }
    }
    __syncthreads();
    const T d = dg[i - k0p];
    for (int c = k0p + tid; c < i; c += PT) u[c - k0p] = D[c] * F[(int64_t)c * f + i];
    __syncthreads();
    // pivot column (rows of F11 below the pivot), left-looking within the panel;
    // each thread keeps its rows in registers so the loads of a column overlap
    T acc[PROWS];
#pragma unroll
    for (int t = 0; t < PROWS; ++t) {
      const int r = i + 1 + tid + t * PT;
      acc[t] = (r < p) ? F[(int64_t)i * f + r] : (T)0;
    }
    for (int c = k0p; c < i; ++c) {
      const T uc = u[c - k0p];
      const T* Fc = F + (int64_t)c * f;
#pragma unroll
      for (int t = 0; t < PROWS; ++t) {
        const int r = i + 1 + tid + t * PT;
        if (r < p) acc[t] -= Fc[r] * uc;
      }
    }
    const T inv = (T)1 / d;
#pragma unroll
    for (int t = 0; t < PROWS; ++t) {
      const int r = i + 1 + tid + t * PT;
      if (r < p) {
        const T l = acc[t] * inv;
        F[(int64_t)i * f + r] = l;
        dg[r - k0p] -= l * acc[t];
      }
    }
    if (tid == 0) {
      F[(int64_t)i * f + i] = d;
      D[i] = d;
    }
    dprev = (double)d;
    have_prev = 1;
    __syncthreads();
  }
  if (tid == 0) {
    NodeState ns;
    ns.npiv = i;
    ns.dprev = dprev;
    ns.done = (i < iend || i == p) ? 1 : 0;
    st[j] = ns;
  }
}

// Row exchanges of the panel at k0p applied to the columns of earlier panels
// (one thread per column, exchanges in pivot order).
template <class T>
__global__ void k_apply_swaps(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
                              const NodeState* __restrict__ st, const int32_t* __restrict__ swaps,
                              T* __restrict__ front, int k0p) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k0p || k0p >= npiv) return;
  const int iend = min(npiv, k0p + PANEL_NB);
  const int32_t* sw = swaps + ni.start;
  T* Fc = front + ni.front_off + (int64_t)c * ni.f;
  for (int i = k0p; i < iend; ++i) {
    const int k = sw[i];
    if (k != i) {
      const T a = Fc[i];
      Fc[i] = Fc[k];
      Fc[k] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric rank-K update C -= A diag(D) A^T on the lower triangle, batched over
// the fronts of a level.  mode 0: trailing F11 update after the panel at k0p;
// mode 1: contribution block F22 -= L21 D L21^T.
// ---------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(256)
k_syrk(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
       const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval, int mode,
       int k0p) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const NodeState s = st[j];
  int r0, kc0, K, nr;
  if (mode == 0) {
    if (s.done || k0p >= ni.p) return;
    r0 = k0p + PANEL_NB;
    kc0 = k0p;
    K = PANEL_NB;
    nr = ni.p - r0;
  } else {
    r0 = ni.p;
    kc0 = 0;
    K = s.npiv;
    nr = ni.b;
  }
  if (nr <= 0 || K <= 0) return;
  // tile (ti, tj), ti >= tj
  const int t = blockIdx.x;
  int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int nt = (nr + 63) / 64;
  if (ti >= nt) return;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  const T* A = F + (int64_t)kc0 * f + r0;  // A(r, k) = A[k*f + r]
  const T* Dk = dval + ni.start + kc0;
  T* C = F + (int64_t)r0 * f + r0;

  __shared__ T As[16][64 + 1];
  __shared__ T Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
  const int rowA = ti * 64, rowB = tj * 64;
  for (int kk = 0; kk < K; kk += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int rr = e & 63, kq = e >> 6;
      const int kg = kk + kq;
      T va = (T)0, vb = (T)0;
      if (kg < K) {
        if (rowA + rr < nr) va = A[(int64_t)kg * f + rowA + rr];
        if (rowB + rr < nr) vb = A[(int64_t)kg * f + rowB + rr] * Dk[kg];
      }
      As[kq][rr] = va;
      Bs[kq][rr] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 16; ++kq) {
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
  for (int x = 0; x < 4; ++x) {
    const int r = rowA + ty * 4 + x;
    if (r >= nr) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = rowB + tx * 4 + y;
      if (c < nr && c <= r) C[(int64_t)c * f + r] -= acc[x][y];
    }
  }
}

// ---------------------------------------------------------------------------
// F3: L21 = F21 L11^{-T} D^{-1}, one workgroup per 64-row strip of F21
// ---------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(256)
k_trsm(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
       const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int b = ni.b;
  const int rs = blockIdx.x * 64;
  if (rs >= b || npiv == 0) return;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  T* X = F + ni.p + rs;  // X(r, c) = X[c*f + r], r < 64
  const int nrow = min(64, b - rs);
  const T* Dk = dval + ni.start;
  __shared__ T As[16][64 + 1];
  __shared__ T Bs[16][64 + 1];
  __shared__ T Xt[64][64 + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int J0 = 0; J0 < npiv; J0 += 64) {
    const int nc = min(64, npiv - J0);
    T acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = (T)0;
    for (int kk = 0; kk < J0; kk += 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + q * 256;
        const int rr = e & 63, kq = e >> 6;
        const int kg = kk + kq;
        As[kq][rr] = (rr < nrow) ? X[(int64_t)kg * f + rr] : (T)0;
        Bs[kq][rr] = (rr < nc) ? F[(int64_t)kg * f + J0 + rr] : (T)0;
      }
      __syncthreads();
#pragma unroll
      for (int kq = 0; kq < 16; ++kq) {
        T a[4], bb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) { a[q] = As[kq][ty * 4 + q]; bb[q] = Bs[kq][tx * 4 + q]; }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * bb[y];
      }
      __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int r = ty * 4 + x, c = tx * 4 + y;
        Xt[r][c] = (r < nrow && c < nc) ? X[(int64_t)(J0 + c) * f + r] - acc[x][y] : (T)0;
      }
    __syncthreads();
    // unit lower triangular solve inside the block (one thread per row)
    if (tid < nrow) {
      for (int c = 1; c < nc; ++c) {
        T v = Xt[tid][c];
        for (int c2 = 0; c2 < c; ++c2) v -= Xt[tid][c2] * F[(int64_t)(J0 + c2) * f + J0 + c];
        Xt[tid][c] = v;
      }
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e & 63, c = e >> 6;
      if (r < nrow && c < nc) X[(int64_t)(J0 + c) * f + r] = Xt[r][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < 64 * npiv; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (r < nrow) X[(int64_t)c * f + r] /= Dk[c];
  }
}

// ---------------------------------------------------------------------------
// hard part: mark every postponed index
// ---------------------------------------------------------------------------

__global__ void k_mark_l2(int32_t n_nodes, const NodeInfo* __restrict__ nodes,
                          const NodeState* __restrict__ st, const int32_t* __restrict__ piv,
                          uint8_t* __restrict__ isl2) {
  const int j = blockIdx.x;
  if (j >= n_nodes) return;
  const NodeInfo ni = nodes[j];
  for (int k = st[j].npiv + threadIdx.x; k < ni.p; k += blockDim.x) isl2[piv[ni.start + k]] = 1;
}

__global__ void k_inverse_pivots(int32_t n_nodes, const NodeInfo* __restrict__ nodes,
                                 const int32_t* __restrict__ piv, int32_t* __restrict__ ipos) {
  const int j = blockIdx.x;
  if (j >= n_nodes) return;
  const NodeInfo ni = nodes[j];
  for (int k = threadIdx.x; k < ni.p; k += blockDim.x) ipos[piv[ni.start + k]] = k;
}

__global__ void k_init_state(int32_t n_nodes, NodeState* st) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_nodes) return;
  NodeState s;
  s.npiv = 0;
  s.done = 0;
  s.dprev = 1.0;
  st[j] = s;
}

__global__ void k_iota(int64_t n, int32_t* a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <class T>
void step1(hf_ctx* ctx, const double* values, hipStream_t s) {
  const int64_t n = ctx->n;
  ctx->d_front.alloc((size_t)ctx->front_elems * sizeof(T));
  ctx->d_state.alloc((size_t)ctx->n_nodes * sizeof(NodeState));
  ctx->d_piv.alloc((size_t)n * sizeof(int32_t));
  ctx->d_swaps.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
  ctx->d_dval.alloc((size_t)n * sizeof(T));
  ctx->d_q.alloc((size_t)n * sizeof(double));
  ctx->d_kval.alloc((size_t)ctx->nnz * sizeof(double));
  ctx->d_kbar.alloc((size_t)ctx->nnz * sizeof(double));
  ctx->d_isl2.alloc((size_t)n);
  ctx->d_flag.alloc(64);
  T* front = ctx->d_front.as<T>();
  const NodeInfo* nodes = ctx->d_nodes.as<NodeInfo>();
  NodeState* st = ctx->d_state.as<NodeState>();
  int* flag = ctx->d_flag.as<int>();
  HF_HIP(hipMemsetAsync(flag, 0, 64, s));
  HF_HIP(hipMemsetAsync(front, 0, (size_t)ctx->front_elems * sizeof(T), s));
  HF_HIP(hipMemsetAsync(ctx->d_isl2.ptr, 0, (size_t)n, s));
  if (n > 0) {
    k_iota<<<cdiv(n, 256), 256, 0, s>>>(n, ctx->d_piv.as<int32_t>());
    k_scale_q<<<cdiv(n, 256), 256, 0, s>>>(n, ctx->d_pindptr.as<int64_t>(), ctx->d_diagpos.as<int32_t>(),
                                           ctx->d_psrc.as<int64_t>(), values, ctx->d_q.as<double>(), flag);
    k_scale_assemble<T><<<cdiv(n, 256), 256, 0, s>>>(
        n, ctx->d_pindptr.as<int64_t>(), ctx->d_pindices.as<int32_t>(), ctx->d_psrc.as<int64_t>(),
        ctx->d_asm.as<int64_t>(), values, ctx->d_q.as<double>(), ctx->d_kval.as<double>(),
        ctx->d_kbar.as<double>(), front, flag);
  }
  k_init_state<<<cdiv(std::max(ctx->n_nodes, 1), 256), 256, 0, s>>>(ctx->n_nodes, st);
  HF_HIP(hipGetLastError());
  int hflag = 0;
  HF_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HF_HIP(hipStreamSynchronize(s));
  if (hflag) throw Status{HF_ERR_VALUE};

  const int nlev = (int)ctx->level_ptr.size() - 1;
  const int32_t* lnodes_all = ctx->d_level_nodes.as<int32_t>();
  KTimer& tm = ctx->timer;
  const double sz = sizeof(T);
  size_t ea = 0;
  for (int l = 0; l < nlev; ++l) {
    const int32_t q0 = ctx->level_ptr[l], q1 = ctx->level_ptr[l + 1];
    const int nl = q1 - q0;
    const int32_t* lnodes = lnodes_all + q0;
    // algorithmic work of a launch over this level (symbolic sizes)
    auto level_sum = [&](auto&& fn) {
      double by = 0.0, fl = 0.0;
      if (!tm.on) return std::make_pair(by, fl);
      for (int32_t q = q0; q < q1; ++q) fn(ctx->nodes[ctx->level_nodes[q]], by, fl);
      return std::make_pair(by, fl);
    };
    // extend-add of the children (one launch per child rank)
    for (; ea < ctx->ea_launch.size() && ctx->ea_launch[ea].level == l; ++ea) {
      const EaLaunch& el = ctx->ea_launch[ea];
      double by = 0.0, fl = 0.0;
      if (tm.on)
        for (int q = 0; q < el.count; ++q) {
          const double b = ctx->nodes[ctx->ea_items[el.off + q]].b;
          by += 1.5 * b * b * sz;
          fl += 0.5 * b * b;
        }
      dim3 grid(cdiv(el.maxb, 16), (unsigned)el.count);
      timed(tm, HF_K_EXTEND_ADD, by, fl, s, [&] {
        k_extend_add<T><<<grid, 256, 0, s>>>(ctx->d_ea_items.as<int32_t>() + el.off, el.count, nodes,
                                             ctx->d_relmap.as<int32_t>(), front);
      });
    }
    // F11 panels
    const int maxp = ctx->level_maxp[l];
    const size_t shm = (size_t)std::max(maxp, 1) * sizeof(T);
    for (int k0p = 0; k0p < maxp; k0p += PANEL_NB) {
      auto w1 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        if (ni.p <= k0p) return;
        const double r = ni.p - k0p, nb = std::min(PANEL_NB, ni.p - k0p);
        by += 2.0 * r * nb * sz;
        fl += nb * nb * r;
      });
      timed(tm, HF_K_PANEL, w1.first, w1.second, s, [&] {
        k_panel<T><<<nl, PT, shm, s>>>(lnodes, nodes, st, front, ctx->d_piv.as<int32_t>(),
                                       ctx->d_swaps.as<int32_t>(), ctx->d_dval.as<T>(), k0p, ctx->opt.tau,
                                       ctx->opt.first_pivot_unit);
        if (k0p > 0) {
          dim3 gs(cdiv(k0p, 256), (unsigned)nl);
          k_apply_swaps<T><<<gs, 256, 0, s>>>(lnodes, nodes, st, ctx->d_swaps.as<int32_t>(), front, k0p);
        }
      });
      const int nr = maxp - (k0p + PANEL_NB);
      if (nr > 0) {
        const int nt = (nr + 63) / 64;
        dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)nl);
        auto w2 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
          const double r = ni.p - k0p - PANEL_NB;
          if (r <= 0) return;
          by += (r * PANEL_NB + r * r) * sz;
          fl += r * r * PANEL_NB;
        });
        timed(tm, HF_K_F11_UPDATE, w2.first, w2.second, s, [&] {
          k_syrk<T><<<grid, 256, 0, s>>>(lnodes, nodes, st, front, ctx->d_dval.as<T>(), 0, k0p);
        });
      }
    }
    // F21, F22
    const int maxb = ctx->level_maxb[l];
    if (maxb > 0) {
      dim3 g1(cdiv(maxb, 64), (unsigned)nl);
      auto w3 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        const double b = ni.b, p = ni.p;
        by += (2.0 * b * p + 0.5 * p * p) * sz;
        fl += b * p * p;
      });
      timed(tm, HF_K_TRSM, w3.first, w3.second, s, [&] {
        k_trsm<T><<<g1, 256, 0, s>>>(lnodes, nodes, st, front, ctx->d_dval.as<T>());
      });
      const int nt = (maxb + 63) / 64;
      dim3 g2((unsigned)(nt * (nt + 1) / 2), (unsigned)nl);
      auto w4 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        const double b = ni.b, p = ni.p;
        by += (b * p + b * b) * sz;
        fl += b * b * p;
      });
      timed(tm, HF_K_SYRK, w4.first, w4.second, s, [&] {
        k_syrk<T><<<g2, 256, 0, s>>>(lnodes, nodes, st, front, ctx->d_dval.as<T>(), 1, 0);
      });
    }
    HF_HIP(hipGetLastError());
  }
  ctx->d_ipos.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
  if (ctx->n_nodes > 0) {
    k_mark_l2<<<ctx->n_nodes, 256, 0, s>>>(ctx->n_nodes, nodes, st, ctx->d_piv.as<int32_t>(),
                                           ctx->d_isl2.as<uint8_t>());
    k_inverse_pivots<<<ctx->n_nodes, 256, 0, s>>>(ctx->n_nodes, nodes, ctx->d_piv.as<int32_t>(),
                                                  ctx->d_ipos.as<int32_t>());
  }
  prepare_solve<T>(ctx, s);
  HF_HIP(hipGetLastError());
}

template void step1<float>(hf_ctx*, const double*, hipStream_t);
template void step1<double>(hf_ctx*, const double*, hipStream_t);

}  // namespace hf
