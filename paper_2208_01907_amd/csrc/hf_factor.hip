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
//   F21 (b x p~): L21 = F21 L11^{-T} D^{-1}  (blocked TRSM: windows of one sweep
//                 step, each a product with the inverse of its diagonal block)
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
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);  // one wave per column of the child block
  if (t >= bc) return;
  const T* C = front + ci.front_off;
  T* F = front + pi.front_off;
  const int32_t* rel = relmap + ci.border_off;
  const int64_t fc = ci.f, fp = pi.f;
  const int64_t ct = (int64_t)(ci.p + t) * fc + ci.p;
  const int64_t pt = (int64_t)rel[t] * fp;
  for (int r = t + (threadIdx.x & 63); r < bc; r += 64) F[pt + rel[r]] += C[ct + r];
}

// ---------------------------------------------------------------------------
// F2: panel factorization of F11 with pivot search and postponing
// ---------------------------------------------------------------------------

constexpr int PT = 512;               // threads of the panel kernel (2 waves per SIMD: 256 VGPRs each)
constexpr int PROWS = 4096 / PT;      // pivot-block rows per thread (nodes hold at most 4096 indices)
// register slots a panel launch needs: the level's largest remaining pivot
// block, rounded up to a power of two times PT
inline int panel_slots(int rem) { return rem <= PT ? 1 : rem <= 2 * PT ? 2 : rem <= 4 * PT ? 4 : PROWS; }

// Panel width: the panel's L values of every pivot-block row stay in registers.
template <class T>
struct PanelWidth {
  static constexpr int value = sizeof(T) == 4 ? 16 : 8;
};
// one row of panel values as a register vector: an element chosen by a
// wave-uniform index is read or written in place (GPR index mode), with no
// select over the whole row
template <class T, int W>
struct PanelRow {
  typedef T V __attribute__((ext_vector_type(W)));
};
// Panels over small remaining blocks (one register slot per thread) take
// twice the pivots: half the trailing updates and panel launches for a
// few more products per pivot.
inline int panel_pivots(int base, int slots) { return slots <= 1 ? 2 * base : base; }

// Wave-wide reductions with DPP row shifts and row broadcasts; the result of
// lane 63 is returned to every lane.  Lanes without a source keep their value.
template <int CTRL, int RM>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, RM, 0xf, false);
}
template <class Op>
__device__ __forceinline__ int wave_reduce_i(int x, Op op) {
  x = op(x, dpp_i<0x111, 0xf>(x));  // row_shr:1
  x = op(x, dpp_i<0x112, 0xf>(x));  // row_shr:2
  x = op(x, dpp_i<0x114, 0xf>(x));  // row_shr:4
  x = op(x, dpp_i<0x118, 0xf>(x));  // row_shr:8
  x = op(x, dpp_i<0x142, 0xa>(x));  // row_bcast:15
  x = op(x, dpp_i<0x143, 0xc>(x));  // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ float wave_max(float v) {
  return __int_as_float(wave_reduce_i(__float_as_int(v), [](int a, int b) {
    return __float_as_int(fmaxf(__int_as_float(a), __int_as_float(b)));
  }));
}
template <int CTRL, int RM>
__device__ __forceinline__ void dmax_step(int& lo, int& hi) {
  const int l2 = dpp_i<CTRL, RM>(lo), h2 = dpp_i<CTRL, RM>(hi);
  const double m = fmax(__hiloint2double(hi, lo), __hiloint2double(h2, l2));
  lo = __double2loint(m);
  hi = __double2hiint(m);
}
__device__ __forceinline__ double wave_max(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  dmax_step<0x111, 0xf>(lo, hi);
  dmax_step<0x112, 0xf>(lo, hi);
  dmax_step<0x114, 0xf>(lo, hi);
  dmax_step<0x118, 0xf>(lo, hi);
  dmax_step<0x142, 0xa>(lo, hi);
  dmax_step<0x143, 0xc>(lo, hi);
  return __hiloint2double(__builtin_amdgcn_readlane(hi, 63), __builtin_amdgcn_readlane(lo, 63));
}
__device__ __forceinline__ int wave_min(int v) {
  return wave_reduce_i(v, [](int a, int b) { return a < b ? a : b; });
}
// the same for an unsigned 64-bit key held as (hi, lo)
template <int CTRL, int RM>
__device__ __forceinline__ void kmax_step(uint64_t& k) {
  const uint32_t h2 = (uint32_t)dpp_i<CTRL, RM>((int)(uint32_t)(k >> 32));
  const uint32_t l2 = (uint32_t)dpp_i<CTRL, RM>((int)(uint32_t)k);
  const uint64_t k2 = ((uint64_t)h2 << 32) | l2;
  k = k2 > k ? k2 : k;
}
__device__ __forceinline__ uint64_t wave_max_key(uint64_t k) {
  kmax_step<0x111, 0xf>(k);
  kmax_step<0x112, 0xf>(k);
  kmax_step<0x114, 0xf>(k);
  kmax_step<0x118, 0xf>(k);
  kmax_step<0x142, 0xa>(k);
  kmax_step<0x143, 0xc>(k);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 63);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)k, 63);
  return ((uint64_t)hi << 32) | lo;
}

// Panel factorization with pivot search and postponing, one workgroup per front.
//
// The trailing block [k0p, p)^2 of the pivot block is stored full (both
// triangles).  A symmetric exchange of positions i and k moves no data: every
// row keeps the storage index ("phys") of its row and column, and the rows
// only exchange their positions.  Thread t holds rows q = t + NT*s (relative to
// k0p, q their position when the panel starts) in registers for the whole
// panel: their panel values L[., 0..NB), current diagonal, nested-dissection
// index, phys and current position.  Per pivot: a wave-wide argmax (DPP) over
// the rows not yet pivoted, each wave posts its candidate (with that row's
// panel values); one barrier; every thread combines the wave records, the
// winner takes position i and the row at position i takes the winner's old
// position (two compares per row), and each thread reads its rows of the pivot
// column (one coalesced column read) and forms the new L column (left-looking
// inside the panel).  The posted copies alternate between two buffers, so a
// buffer is rewritten only after every thread has passed the next barrier.
// At the end, every row is written at its final position: the storage index of
// every trailing position goes to `physmap` (k_trail_update reads its source
// tiles through it; no storage column moves), the panel's L columns go to the
// side buffer `lbuf` in position order, and a snapshot of the position -> index
// map is kept for k_l11_gather.
template <class T, int PR, int NB, int NT = PT>
__global__ void __launch_bounds__(NT)
k_panel(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes, NodeState* st,
        T* __restrict__ front, int32_t* __restrict__ piv, int32_t* __restrict__ snap,
        T* __restrict__ dval, int32_t* __restrict__ physmap, T* __restrict__ lbuf, int k0p, double tau,
        int first_unit) {
  constexpr int NB0 = PanelWidth<T>::value;  // snapshot granularity
  static_assert(NB == NB0 || NB == 2 * NB0, "panel width");
  constexpr int NW = NT / 64;  // waves (NT < PT for blocks of at most NT rows)
  const int j = lnodes[blockIdx.x];
  const NodeInfo ni = nodes[j];
  const NodeState s0 = st[j];
  if (s0.done || k0p >= ni.p || ni.p - k0p > PR * NT) return;  // the launch sizes PR, NT for the level
  const int p = ni.p;
  const uint32_t f = (uint32_t)ni.f;  // fronts hold fewer than 2^31 entries (checked at analysis)
  T* F = front + ni.front_off;
  T* Fb = F + (uint32_t)k0p * f + k0p;  // trailing block: Fb[c*f + r], r, c relative to k0p
  int32_t* idx_g = piv + ni.start;
  T* D = dval + ni.start;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int P = p - k0p;

  // one record per wave: |d|, d, index, position, storage index of its candidate
  struct alignas(16) WaveRec {
    T v, d;
    int id, k, ph;
  };
  __shared__ WaveRec rec[2][NW];
  __shared__ __align__(64) T pubK[2][NW][NB];  // panel row of each wave's candidate
  using Row = typename PanelRow<T, NB>::V;

  Row Lp[PR];
  Row Dlr = (Row)((T)0);
  T dgr[PR];
  int idxr[PR], ph[PR], pos[PR];
  // FP32: the argmax key of a row, (bits of |d|) * 2^32 + (2^32 - 1 - index),
  // orders rows as (larger |d|, then smaller index); 0 for rows out of the race
  uint64_t key[PR];
#pragma unroll
  for (int s = 0; s < PR; ++s) {
    const int q = tid + NT * s;
    Lp[s] = (Row)((T)0);
    dgr[s] = (T)0;
    idxr[s] = INT_MAX;
    ph[s] = q;
    pos[s] = q;  // padding rows (q >= P) never move
    if (q < P) {
      dgr[s] = Fb[(uint32_t)q * f + q];
      idxr[s] = idx_g[k0p + q];
    }
    key[s] = 0;
    if constexpr (sizeof(T) == 4)
      if (q < P) key[s] = ((uint64_t)__float_as_uint(fabsf((float)dgr[s])) << 32) | (uint32_t)~idxr[s];
  }
  if (tid < 2 * NW) {  // defined contents even if a wave posted nothing
    WaveRec r0;
    r0.v = (T)-1;
    r0.d = (T)0;
    r0.id = INT_MAX;
    r0.k = 0;
    r0.ph = 0;
    rec[tid / NW][tid % NW] = r0;
  }
  __syncthreads();
  double dprev = s0.dprev;
  double dstop = s0.dstop;
  int have_prev = (s0.npiv > 0) ? 1 : first_unit;
  const int iend = min(k0p + NB, p);
  int i;
  for (i = k0p; i < iend; ++i) {
    const int qi = i - k0p;
    const int par = qi & 1;
    // own best candidate: max |diag|, ties to the smallest index
    T av = (T)-1, wmax;
    int aid = INT_MAX, as = -1, wid;
    if constexpr (sizeof(T) == 4) {  // one 64-bit key per row, one reduction
      uint64_t bk = 0;
#pragma unroll
      for (int s = 0; s < PR; ++s) {
        const bool better = key[s] > bk;
        bk = better ? key[s] : bk;
        as = better ? s : as;
      }
      const uint64_t wk = wave_max_key(bk);
      wmax = wk ? (T)__uint_as_float((uint32_t)(wk >> 32)) : (T)-1;
      wid = (int)~(uint32_t)wk;
      av = (bk == wk && wk) ? wmax : (T)-1;
      aid = wid;
    } else {
#pragma unroll
      for (int s = 0; s < PR; ++s) {  // branch-free: bitwise tests and selects
        const T v = (pos[s] >= qi && pos[s] < P) ? fabs(dgr[s]) : (T)-1;
        const bool better = (v > av) | ((v == av) & (idxr[s] < aid));
        av = better ? v : av;
        aid = better ? idxr[s] : aid;
        as = better ? s : as;
      }
      wmax = wave_max(av);
      wid = wave_min(av == wmax ? aid : INT_MAX);
    }
    if (wmax >= (T)0 && av == wmax && aid == wid) {  // the wave's winner posts its row
      const int asu = __builtin_amdgcn_readfirstlane(as);  // one lane: uniform here
#pragma unroll
      for (int s = 0; s < PR; ++s)
        if (s == asu) {
          *reinterpret_cast<Row*>(pubK[par][wv]) = Lp[s];
          WaveRec r1;
          r1.v = wmax;
          r1.d = dgr[s];
          r1.id = wid;
          r1.k = pos[s];
          r1.ph = ph[s];
          rec[par][wv] = r1;
        }
    }
    if (lane == 0 && wmax < (T)0) {  // no candidate in this wave
      WaveRec r1;
      r1.v = (T)-1;
      r1.d = (T)0;
      r1.id = INT_MAX;
      r1.k = 0;
      r1.ph = 0;
      rec[par][wv] = r1;
    }
    __syncthreads();
    // the wave records, read together, then combined without branches
    WaveRec rw[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) rw[w] = rec[par][w];
    // the winner's fields are selected in registers along the way (no second
    // LDS round trip for them)
    int ww = 0;
    WaveRec best = rw[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const bool g = (rw[w].v > best.v) | ((rw[w].v == best.v) & (rw[w].id < best.id));
      best.v = g ? rw[w].v : best.v;
      best.d = g ? rw[w].d : best.d;
      best.id = g ? rw[w].id : best.id;
      best.k = g ? rw[w].k : best.k;
      best.ph = g ? rw[w].ph : best.ph;
      ww = g ? w : ww;
    }
    ww = __builtin_amdgcn_readfirstlane(ww);
    const int bid = best.id;
    const Row rowK = *reinterpret_cast<const Row*>(pubK[par][ww]);  // panel row of the pivot row
    const int qk = min(max(best.k, qi), P - 1);
    const T d = best.d;
    const int phK = min(max(best.ph, 0), P - 1);
    const double dk = (double)d;
    bool stop = (dk == 0.0);
    if (!stop && have_prev && fabs(dk) < tau * fabs(dprev)) stop = true;
    if (stop) {  // uniform: every thread computed the same decision
      dstop = dk;
      break;
    }
    // positions i and k exchange their rows: the winner takes position i, the
    // row at position i takes the winner's position
#pragma unroll
    for (int s = 0; s < PR; ++s) pos[s] = (idxr[s] == bid) ? qi : (pos[s] == qi ? qk : pos[s]);
    // u_c = D_c L[i, c] for the panel columns so far (the pivot row); the
    // pivots of later columns are still zero, as are the row's later values
    const Row u = Dlr * rowK;
    Dlr[qi] = d;  // every thread keeps the panel's pivots
    const T inv = (T)1 / d;
    // the pivot column: storage column phK at the storage rows of the rows
    const T* colK = Fb + (uint32_t)phK * f;
    T v[PR];
#pragma unroll
    for (int s = 0; s < PR; ++s) v[s] = (pos[s] > qi && pos[s] < P) ? colK[ph[s]] : (T)0;
    // left-looking column: only the qi columns factored so far contribute
    // (qi is uniform, so the cut is a scalar branch)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < qi) {
#pragma unroll
        for (int s = 0; s < PR; ++s) v[s] -= Lp[s][c] * u[c];
      }
    }
    // rows at or before the pivot position and padding rows keep zeros in the
    // new column; their diagonals are never read again
#pragma unroll
    for (int s = 0; s < PR; ++s) {
      const bool live = (pos[s] > qi) & (pos[s] < P);
      const T l = live ? v[s] * inv : (T)0;
      dgr[s] -= l * v[s];
      Lp[s][qi] = l;
      if constexpr (sizeof(T) == 4)  // the rows still in the race for the next pivot
        key[s] = live ? ((uint64_t)__float_as_uint(fabsf((float)dgr[s])) << 32) | (uint32_t)~idxr[s] : 0;
    }
    dprev = dk;
    have_prev = 1;
  }
  const int nacc = i - k0p;
  // the panel's pivots
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (tid == c && c < nacc) D[k0p + c] = Dlr[c];
  // storage index of every trailing position (k_trail_update resolves the
  // exchanges from it; the panel's storage columns keep their values until then)
  int32_t* pm = physmap + ni.start + k0p;
#pragma unroll
  for (int s = 0; s < PR; ++s)
    if (pos[s] >= nacc && pos[s] < P) pm[pos[s]] = ph[s];
  // the panel's L columns, in position order, to the side buffer; the snapshot
  // of the position -> index map
  T* Lb = lbuf + ni.lbuf_off + (int64_t)k0p * ni.lbuf_ld + k0p;  // Lb[c*ld + q]
  int32_t* sn = snap + ni.snap_off + (int64_t)(k0p / NB0) * p;  // a wide panel fills two slots
#pragma unroll
  for (int s = 0; s < PR; ++s) {
    const int q = pos[s];
    if (q < P) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nacc && c < q) Lb[(int64_t)c * ni.lbuf_ld + q] = Lp[s][c];
      idx_g[k0p + q] = idxr[s];
      sn[k0p + q] = idxr[s];
      if constexpr (NB == 2 * NB0)  // the second half's slot, where that half has columns
        if (k0p + NB0 < p) sn[p + k0p + q] = idxr[s];
    }
  }
  if (tid == 0) {
    NodeState ns;
    ns.npiv = i;
    ns.dprev = dprev;
    ns.dstop = dstop;
    ns.done = (i < iend || i == p) ? 1 : 0;
    st[j] = ns;
  }
}

// Full (both triangles) storage of the pivot block before its first panel:
// the upper triangle receives the transpose of the assembled lower triangle.
template <class T>
__global__ void __launch_bounds__(256)
k_mirror(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes, T* __restrict__ front) {
  const int j = lnodes[blockIdx.z];
  const NodeInfo ni = nodes[j];
  const int p = ni.p;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;  // lower tile rows r0.., columns c0..
  if (r0 >= p || c0 >= p || r0 + 63 < c0) return;
  const uint32_t f = (uint32_t)ni.f;
  T* F = front + ni.front_off;
  __shared__ T tile[64][65];
  const int tid = threadIdx.x, l = tid & 63;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int cc = (tid >> 6) + 4 * q;
    const int r = r0 + l, c = c0 + cc;
    if (r < p && c < r) tile[cc][l] = F[(uint32_t)c * f + r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = (tid >> 6) + 4 * q;
    const int r = r0 + rr, c = c0 + l;
    if (r < p && c < r) F[(uint32_t)r * f + c] = tile[l][rr];
  }
}

// Trailing update after the panel at k0p, with the exchanges of the panel
// resolved: T'(x, y) = A(x, y) - sum_t L[x, t] D_t L[y, t] for positions
// x, y >= k0p + NB, A(x, y) = storage(phys x, phys y), read from the scratch
// copy of the storage column when x or y is displaced (by symmetry a storage
// column is also a storage row).  Lower tiles are computed; each result is
// written to both triangles.  Reads of the storage in place touch only
// non-displaced entries of the tile itself, so updating in place is safe.
template <class T, int NB, int H16 = 0>
__global__ void __launch_bounds__(256)
k_trail_update(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
               const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval,
               const int32_t* __restrict__ physmap, const T* __restrict__ lbuf, int k0p) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const NodeState sj = st[j];
  if (sj.done || k0p >= ni.p) return;
  const int r0 = NB;  // relative to k0p
  const int P = ni.p - k0p;
  const int nr = P - r0;
  if (nr <= 0) return;
  const int t = blockIdx.x;
  int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int nt = (nr + 63) / 64;
  if (ti >= nt) return;
  const uint32_t f = (uint32_t)ni.f;
  T* Fb = front + ni.front_off + (uint32_t)k0p * f + k0p;
  const T* Dk = dval + ni.start + k0p;
  const int32_t* pm = physmap + ni.start + k0p;
  const T* Lb = lbuf + ni.lbuf_off + (int64_t)k0p * ni.lbuf_ld + k0p;  // L[q, c] = Lb[c*ld + q]
  const int64_t ldl = ni.lbuf_ld;

  __shared__ T As[16][64 + 4];
  __shared__ T Bs[16][64 + 4];
  __shared__ int phx[64], phy[64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int rowA = r0 + ti * 64, rowB = r0 + tj * 64;
  if (tid < 64) {
    const int x = rowA + tid;
    phx[tid] = x < P ? pm[x] : 0;
  } else if (tid < 128) {
    const int y = rowB + tid - 64;
    phy[tid - 64] = y < P ? pm[y] : 0;
  }
  __syncthreads();
  // the old values first (their loads overlap the product below)
  T old[2][2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int ly = wr + bi * 16 + Mfma<T>::row(lane, tt);
        const int lx = wc + bj * 16 + (lane & 15);  // lane-fast: the storage row
        const int x = rowA + lx, y = rowB + ly;
        T a = (T)0;
        // A(x, y) = storage(phys x, phys y): a displaced position's storage is a
        // column of the panel, which this kernel never writes
        if (x < P && y < P && y <= x) a = Fb[(uint32_t)phy[ly] * f + phx[lx]];
        old[bi][bj][tt] = a;
      }
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
  __shared__ float smx[2][4];  // FP16 products: per-stage operand maxima of the four waves
  for (int kk = 0; kk < NB; kk += 16) {
    float ma = 0.f, mb = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int rr = e & 63, kq = e >> 6;
      const int kg = kk + kq;
      T va = (T)0, vb = (T)0;
      if (kg < NB) {
        if (rowA + rr < P) va = Lb[kg * ldl + rowA + rr];
        if (rowB + rr < P) vb = Lb[kg * ldl + rowB + rr] * Dk[kg];
      }
      As[kq][rr] = vb;  // the product is formed transposed: rows of the tile on the lanes
      Bs[kq][rr] = va;
      if constexpr (H16 > 0) {
        ma = fmaxf(ma, fabsf((float)vb));
        mb = fmaxf(mb, fabsf((float)va));
      }
    }
    if constexpr (H16 > 0) {
      stage_max_post(ma, smx[0], lane, w);
      stage_max_post(mb, smx[1], lane, w);
    }
    __syncthreads();
    if constexpr (H16 > 0)
      mfma_tile_64_h16<68, H16 == 2>(As, Bs, acc, lane, wr, wc, fp16_scale(stage_max_read(smx[0])),
                                     fp16_scale(stage_max_read(smx[1])));
    else
      mfma_tile_64<T, 16, 68>(As, Bs, acc, lane, wr, wc);
    __syncthreads();
  }
  // lower triangle straight from the product layout (lanes along storage rows);
  // the mirror goes through LDS so that its stores also run along storage rows
  __shared__ T mt[64][65];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int ly = wr + bi * 16 + Mfma<T>::row(lane, tt);
        const int lx = wc + bj * 16 + (lane & 15);  // lane-fast: the storage row
        const int x = rowA + lx, y = rowB + ly;
        const T v = old[bi][bj][tt] - acc[bi][bj][tt];
        mt[lx][ly] = v;
        if (x < P && y < P && y <= x) Fb[(uint32_t)y * f + x] = v;
      }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int lx = (tid >> 6) + 4 * q, ly = tid & 63;
    const int x = rowA + lx, y = rowB + ly;
    if (x < P && y < P && y <= x) Fb[(uint32_t)x * f + y] = mt[lx][ly];
  }
}

// Once a node is finished, the columns of every panel are put in pivot order:
// the L value of final row a in column c (panel jp) sits at the position that
// the index piv[a] had when panel jp ended.  One workgroup per panel; the
// result goes transposed into the unused upper triangle (k_l11_back copies it
// down), so that no value is overwritten before it is read.
template <class T>
__global__ void __launch_bounds__(256)
k_l11_gather(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, const int32_t* __restrict__ piv,
             const int32_t* __restrict__ snap, const T* __restrict__ lbuf, T* __restrict__ front) {
  constexpr int NB = PanelWidth<T>::value;
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int c0 = blockIdx.x * NB;
  if (c0 >= npiv) return;
  const int p = ni.p;
  const uint32_t f = (uint32_t)ni.f;
  T* F = front + ni.front_off;
  const int32_t* sn = snap + ni.snap_off + (int64_t)blockIdx.x * p;
  const int32_t* pv = piv + ni.start;
  __shared__ int32_t inv[4096];
  for (int x = c0 + threadIdx.x; x < p; x += 256) inv[sn[x] - ni.start] = x;
  __syncthreads();
  const int nc = min(NB, npiv - c0);
  const int rows = npiv - c0;
  for (int e = threadIdx.x; e < rows * NB; e += 256) {
    const int a = c0 + e / NB, cc = e % NB;
    const int c = c0 + cc;
    if (cc < nc && a > c) {
      const int x = inv[pv[a] - ni.start];
      F[(uint32_t)a * f + c] = lbuf[ni.lbuf_off + (int64_t)c * ni.lbuf_ld + x];
    }
  }
}

// L[a, c] = U[c, a] for c < a < npiv (64 x 64 tiles through LDS)
template <class T>
__global__ void __launch_bounds__(256)
k_l11_back(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
           const NodeState* __restrict__ st, const T* __restrict__ dval, T* __restrict__ front) {
  const int j = lnodes[blockIdx.z];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int a0 = blockIdx.x * 64, c0 = blockIdx.y * 64;  // rows a, columns c of L
  if (a0 >= npiv || c0 >= npiv || a0 + 63 < c0) return;
  const uint32_t f = (uint32_t)ni.f;
  T* F = front + ni.front_off;
  __shared__ T tile[64][65];
  const int tid = threadIdx.x, l = tid & 63;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int aa = (tid >> 6) + 4 * q;  // U[c0 + l, a0 + aa] read along c
    const int a = a0 + aa, c = c0 + l;
    if (a < npiv && c < a) tile[aa][l] = F[(uint32_t)a * f + c];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int cc = (tid >> 6) + 4 * q;  // L[a0 + l, c0 + cc] written along a
    const int a = a0 + l, c = c0 + cc;
    if (a < npiv && c < a) F[(uint32_t)c * f + a] = tile[l][cc];
    if (a < npiv && c == a) F[(uint32_t)c * f + a] = dval[ni.start + a];
  }
}

// ---------------------------------------------------------------------------
// Contribution block F22 -= L21 D L21^T (lower triangle), batched over the
// fronts of a level, one 64x64 tile per workgroup.
// ---------------------------------------------------------------------------

template <class T, int H16 = 0>
__global__ void __launch_bounds__(256)
k_syrk(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
       const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval) {
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int r0 = ni.p, kc0 = 0, K = st[j].npiv, nr = ni.b;
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

  __shared__ T As[16][64 + 4];
  __shared__ T Bs[16][64 + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
  const int rowA = ti * 64, rowB = tj * 64;
  __shared__ float smx[2][4];  // FP16 products: per-stage operand maxima of the four waves
  for (int kk = 0; kk < K; kk += 16) {
    float ma = 0.f, mb = 0.f;
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
      As[kq][rr] = vb;  // the product is formed transposed: rows of C on the lanes
      Bs[kq][rr] = va;
      if constexpr (H16 > 0) {
        ma = fmaxf(ma, fabsf((float)vb));
        mb = fmaxf(mb, fabsf((float)va));
      }
    }
    if constexpr (H16 > 0) {
      stage_max_post(ma, smx[0], lane, w);
      stage_max_post(mb, smx[1], lane, w);
    }
    __syncthreads();
    if constexpr (H16 > 0)
      mfma_tile_64_h16<68, H16 == 2>(As, Bs, acc, lane, wr, wc, fp16_scale(stage_max_read(smx[0])),
                                     fp16_scale(stage_max_read(smx[1])));
    else
      mfma_tile_64<T, 16, 68>(As, Bs, acc, lane, wr, wc);
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = rowB + wr + bi * 16 + Mfma<T>::row(lane, t);
        const int r = rowA + wc + bj * 16 + (lane & 15);
        if (r < nr && c < nr && c <= r) C[(int64_t)c * f + r] -= acc[bi][bj][t];
      }
}

// The same product for large borders: 128 x 128 tiles of C per workgroup (each
// wave 64 x 64, 4 x 4 blocks of 16 x 16), half the operand traffic per flop of
// the 64 x 64 tiles.  The operands of stage s+1 (32 values of k) are fetched
// into registers while the matrix cores work on stage s, and the LDS stages
// alternate between two buffers (one barrier per stage).  Every element of C
// accumulates the same products in the same order as in k_syrk (four values of
// k per product, in order), so the results are identical.
template <class T>
__global__ void __launch_bounds__(256)
k_syrk128(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
          const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval) {
  constexpr int KS = 32, LDT = 128 + 4, NQ = KS * 128 / 256;
  const int j = lnodes[blockIdx.y];
  const NodeInfo ni = nodes[j];
  const int r0 = ni.p, K = st[j].npiv, nr = ni.b;
  if (nr <= 0 || K <= 0) return;
  const int t = blockIdx.x;
  int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int nt = (nr + 127) / 128;
  if (ti >= nt) return;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  const T* A = F + r0;  // A(r, k) = A[k*f + r]
  const T* Dk = dval + ni.start;
  T* C = F + (int64_t)r0 * f + r0;
  __shared__ T As[2][KS][LDT];
  __shared__ T Bs[2][KS][LDT];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int rowA = ti * 128, rowB = tj * 128;
  typename Mfma<T>::V acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
  // thread e = tid + 256 q stages row e & 127 of k-value kk + (e >> 7).  The
  // loads are unconditional (indices clamped into the front) so that they all
  // stay in flight; out-of-range values are zeroed when they are staged.
  T ra[NQ], rb[NQ], rd[NQ];
  int kfet = 0;
  auto fetch = [&](int kk) {
    kfet = kk;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + q * 256;
      const int rr = e & 127, kc = min(kk + (e >> 7), K - 1);
      ra[q] = A[(int64_t)kc * f + min(rowA + rr, nr - 1)];
      rb[q] = A[(int64_t)kc * f + min(rowB + rr, nr - 1)];
      rd[q] = Dk[kc];
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + q * 256;
      const int rr = e & 127;
      const bool kin = kfet + (e >> 7) < K;
      const T va = (kin && rowA + rr < nr) ? ra[q] : (T)0;
      const T vb = (kin && rowB + rr < nr) ? rb[q] * rd[q] : (T)0;
      As[buf][e >> 7][rr] = vb;  // transposed product: rows of C on the lanes
      Bs[buf][e >> 7][rr] = va;
    }
  };
  fetch(0);
  stage(0);
  __syncthreads();
  int buf = 0;
  for (int kk = 0; kk < K; kk += KS) {
    const bool more = kk + KS < K;
    if (more) fetch(kk + KS);
#pragma unroll
    for (int k4 = 0; k4 < KS; k4 += 4) {
      const int k = k4 + (lane >> 4);
      T a[4], b[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) a[bi] = As[buf][k][wr + bi * 16 + (lane & 15)];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) b[bj] = Bs[buf][k][wc + bj * 16 + (lane & 15)];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mfma<T>::mma(a[bi], b[bj], acc[bi][bj]);
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = rowB + wr + bi * 16 + Mfma<T>::row(lane, u);
        const int r = rowA + wc + bj * 16 + (lane & 15);
        if (r < nr && c < nr && c <= r) C[(int64_t)c * f + r] -= acc[bi][bj][u];
      }
}

// ---------------------------------------------------------------------------
// F3: L21 = F21 L11^{-T} D^{-1}, one workgroup per 64-row strip of F21
// ---------------------------------------------------------------------------

// The panels leave the border rows of a front in assembly order.  Once the
// node's pivots are final, the border block is gathered in pivot order and
// transposed into the unused upper block of the front:
// G(c, r) = F[(p + r) * f + c] = F21[r, pi(c)], pi(c) the assembly position
// of the index pivoted at c.  The TRSM reads its right-hand side from G.
template <class T>
__global__ void __launch_bounds__(256)
k_gather_border(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
                const NodeState* __restrict__ st, const int32_t* __restrict__ piv, T* __restrict__ front) {
  const int j = lnodes[blockIdx.z];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  if (c0 >= npiv || r0 >= ni.b) return;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  __shared__ T tile[64][65];
  const int tid = threadIdx.x;
  const int lr = tid & 63;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int lc = (tid >> 6) + 4 * q;
    const int c = c0 + lc, r = r0 + lr;
    if (c < npiv && r < ni.b) {
      const int src = piv[ni.start + c] - ni.start;
      tile[lc][lr] = F[(int64_t)src * f + ni.p + r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int lrr = (tid >> 6) + 4 * q, lcc = tid & 63;
    const int c = c0 + lcc, r = r0 + lrr;
    if (c < npiv && r < ni.b) F[(int64_t)(ni.p + r) * f + c] = tile[lcc][lrr];
  }
}

// L21 for the columns of one sweep step [j0, j0 + nc):
// X(r, c) = sum_{k <= c} Y(r, k) Linv(c, k) / D_c, with Y the step's right-hand
// side in G (the contribution of the columns left of the step already removed)
// and Linv the inverse of the step's unit-lower diagonal block.  64x64 tiles of
// (border rows, step columns); the tile goes through LDS so that the columns of
// L21 are written along their rows.
template <class T, int KB>
__global__ void __launch_bounds__(256)
k_trsm_apply(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
             const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval,
             const int64_t* __restrict__ linv2_off, const T* __restrict__ linv2, int j0) {
  constexpr int TB = HF_SWEEP_STEP;
  const int j = lnodes[blockIdx.z];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int rs = blockIdx.x * 64, cs = blockIdx.y * 64;
  if (rs >= ni.b || j0 + cs >= npiv) return;
  const int nc = min(TB, npiv - j0);
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  const T* Li = linv2 + linv2_off[j] + (int64_t)(j0 / TB) * TB * TB;  // Linv(c, k) = Li[k*TB + c]
  const T* Y = F + (int64_t)(ni.p + rs) * f + j0;                     // Y(r, k) = Y[r*f + k]
  const T* Dk = dval + ni.start + j0 + cs;
  const int nrow = min(64, ni.b - rs), ncol = min(64, nc - cs);
  __shared__ T As[KB][68];
  __shared__ T Bs[KB][68];
  __shared__ T Ot[64][65];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
  tile_gemm_64<T, KB, 68, true>(
      acc, As, Bs, 0, min(nc, cs + 64), [&](int k, int r) { return r < nrow ? Y[(int64_t)r * f + k] : (T)0; },
      [&](int k, int c) { return c < ncol ? Li[(int64_t)k * TB + cs + c] : (T)0; }, tid, lane, wr, wc);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = wr + bi * 16 + Mfma<T>::row(lane, t);
        const int c = wc + bj * 16 + (lane & 15);
        Ot[c][r] = (c < ncol) ? acc[bi][bj][t] / Dk[c] : (T)0;
      }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;
    if (r < nrow && c < ncol) F[(int64_t)(j0 + cs + c) * f + ni.p + rs + r] = Ot[c][r];
  }
}

// Blocked TRSM, the part outside the current window of columns [j0, j0 + w):
// G(c, r) -= sum_{k < j0} L21[r, k] D_k L11[c, k] for c in the window, i.e. the
// contribution of the columns already solved (L21 final, so D is put back).
template <class T, int KB>
__global__ void __launch_bounds__(256)
k_trsm_gemm(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
            const NodeState* __restrict__ st, T* __restrict__ front, const T* __restrict__ dval, int j0) {
  const int j = lnodes[blockIdx.z];
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int rs = blockIdx.x * 64;
  const int cs = j0 + blockIdx.y * 64;
  if (rs >= ni.b || cs >= npiv) return;
  const int64_t f = ni.f;
  T* F = front + ni.front_off;
  const T* L21 = F + ni.p + rs;   // L21(r, k) = L21[k*f + r]
  const T* L11 = F + cs;          // L11(c, k) = L11[k*f + c]
  const T* Dk = dval + ni.start;
  T* G = F + (int64_t)(ni.p + rs) * f + cs;  // G(c, r) = G[r*f + c]
  const int nrow = min(64, ni.b - rs), ncol = min(64, npiv - cs);
  __shared__ T As[KB][68];
  __shared__ T Bs[KB][68];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  typename Mfma<T>::V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mfma<T>::V{0, 0, 0, 0};
  tile_gemm_64<T, KB, 68, false>(
      acc, As, Bs, 0, j0, [&](int k, int r) { return r < nrow ? L21[(int64_t)k * f + r] : (T)0; },
      [&](int k, int c) { return c < ncol ? L11[(int64_t)k * f + c] * Dk[k] : (T)0; }, tid, lane, wr, wc);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = wr + bi * 16 + Mfma<T>::row(lane, t);
        const int c = wc + bj * 16 + (lane & 15);
        if (r < nrow && c < ncol) G[(int64_t)r * f + c] -= acc[bi][bj][t];
      }
}

// inverse of every 64x64 unit-lower diagonal block of L11 (one workgroup per block)
template <class T>
__global__ void __launch_bounds__(256)
k_inv_diag(const int32_t* __restrict__ lnodes, const NodeInfo* __restrict__ nodes,
           const NodeState* __restrict__ st, const T* __restrict__ front,
           const int64_t* __restrict__ linv_off, T* __restrict__ linv) {
  const int j = lnodes[blockIdx.y];
  const int B = blockIdx.x;
  const NodeInfo ni = nodes[j];
  const int npiv = st[j].npiv;
  const int J0 = B * 64;
  if (J0 >= npiv) return;
  const int nc = min(64, npiv - J0);
  const int64_t f = ni.f;
  const T* F = front + ni.front_off;
  __shared__ T Ls[64][64 + 1];
  __shared__ T Xs[64][64 + 1];  // Xs[r][c]: column c of the inverse (one thread each)
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    T v = (r == c) ? (T)1 : (T)0;
    if (r > c && r < nc) v = F[(int64_t)(J0 + c) * f + J0 + r];
    Ls[r][c] = v;
    Xs[r][c] = (r == c) ? (T)1 : (T)0;
  }
  __syncthreads();
  if (tid < 64) {  // forward substitution down column c
    const int c = tid;
    for (int r = c + 1; r < 64; ++r) {
      T v = (T)0;
      for (int t = c; t < r; ++t) v -= Ls[r][t] * Xs[t][c];
      Xs[r][c] = v;
    }
  }
  __syncthreads();
  T* out = linv + linv_off[j] + (int64_t)B * 64 * 64;  // column-major 64x64
  for (int e = tid; e < 64 * 64; e += 256) out[e] = Xs[e & 63][e >> 6];
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
  s.dstop = __builtin_nan("");
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
  // FP32 fronts whose two update products run on the FP16 matrix cores: single
  // FP16 operands (1) or FP16 pairs (2)
  const int h16 = sizeof(T) != 4 ? 0
                  : ctx->opt.low_precision == HF_PREC_FP16 ? 1
                  : ctx->opt.low_precision == HF_PREC_FP16_PAIR ? 2 : 0;
  ctx->d_front.alloc((size_t)ctx->front_elems * sizeof(T));
  ctx->d_state.alloc((size_t)ctx->n_nodes * sizeof(NodeState));
  ctx->d_piv.alloc((size_t)n * sizeof(int32_t));
  ctx->d_snap.alloc((size_t)std::max<int64_t>(ctx->snap_elems, 1) * sizeof(int32_t));
  ctx->d_physmap.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
  ctx->d_lbuf.alloc((size_t)std::max<int64_t>(ctx->lbuf_elems, 1) * sizeof(T));
  ctx->d_linv.alloc((size_t)std::max<int64_t>(ctx->linv_elems, 1) * sizeof(T));
  ctx->d_linv2.alloc((size_t)std::max<int64_t>(ctx->linv2_elems, 1) * sizeof(T));
  ctx->d_ninv.alloc((size_t)std::max<int64_t>(ctx->ninv_elems, 1) * sizeof(T));
  ctx->d_ninv_bad.alloc((size_t)std::max(ctx->n_nodes, 1) * sizeof(int32_t));
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
      dim3 grid(cdiv(el.maxb, 4), (unsigned)el.count);
      launch_timed(tm, HF_K_EXTEND_ADD, by, fl, s, k_extend_add<T>, grid, dim3(256),
                   (const int32_t*)(ctx->d_ea_items.as<int32_t>() + el.off), el.count, nodes,
                   (const int32_t*)ctx->d_relmap.as<int32_t>(), front);
    }
    // F11 panels
    constexpr int NBP = PanelWidth<T>::value;
    const int maxp = ctx->level_maxp[l];
    if (maxp > 1) {
      dim3 gm(cdiv(maxp, 64), cdiv(maxp, 64), (unsigned)nl);
      launch_timed(tm, HF_K_OTHER, 0.0, 0.0, s, k_mirror<T>, gm, dim3(256), lnodes, nodes, front);
    }
    for (int k0p = 0, NBL = NBP; k0p < maxp; k0p += NBL) {
      const int slots = panel_slots(maxp - k0p);
      NBL = panel_pivots(NBP, slots);
      auto w1 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        if (ni.p <= k0p) return;
        const double r = ni.p - k0p, nb = std::min(NBL, ni.p - k0p);
        by += 2.0 * r * nb * sz;
        fl += nb * nb * r;
      });
      // blocks of at most 256 / 128 / 64 rows: as many threads (fewer waves to combine)
      const int rem = maxp - k0p;
      const int nt = slots > 1 ? PT : rem <= 64 ? 64 : rem <= 128 ? 128 : rem <= 256 ? 256 : PT;
      auto kp = slots == 1   ? (nt == 64    ? k_panel<T, 1, 2 * NBP, 64>
                                : nt == 128 ? k_panel<T, 1, 2 * NBP, 128>
                                : nt == 256 ? k_panel<T, 1, 2 * NBP, 256>
                                            : k_panel<T, 1, 2 * NBP>)
                : slots == 2 ? k_panel<T, 2, NBP>
                : slots == 4 ? k_panel<T, 4, NBP>
                             : k_panel<T, PROWS, NBP>;
      launch_timed(tm, HF_K_PANEL, w1.first, w1.second, s, kp, dim3((unsigned)nl), dim3(nt), lnodes, nodes,
                   st, front, ctx->d_piv.as<int32_t>(), ctx->d_snap.as<int32_t>(), ctx->d_dval.as<T>(),
                   ctx->d_physmap.as<int32_t>(), ctx->d_lbuf.as<T>(), k0p, ctx->opt.tau,
                   (int)ctx->opt.first_pivot_unit);
      const int nr = maxp - (k0p + NBL);
      if (nr > 0) {
        const int nt = (nr + 63) / 64;
        dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)nl);
        auto w2 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
          const double r = ni.p - k0p - NBL;
          if (r <= 0) return;
          by += (r * NBL + r * r) * sz;
          fl += r * r * NBL;
        });
        constexpr int H1 = sizeof(T) == 4 ? 1 : 0, H2 = sizeof(T) == 4 ? 2 : 0;
        auto ku = NBL == NBP ? (h16 == 1 ? k_trail_update<T, NBP, H1>
                                : h16 == 2 ? k_trail_update<T, NBP, H2> : k_trail_update<T, NBP>)
                             : (h16 == 1 ? k_trail_update<T, 2 * NBP, H1>
                                : h16 == 2 ? k_trail_update<T, 2 * NBP, H2> : k_trail_update<T, 2 * NBP>);
        launch_timed(tm, HF_K_F11_UPDATE, w2.first, w2.second, s, ku, grid, dim3(256), lnodes, nodes,
                     (const NodeState*)st, front, (const T*)ctx->d_dval.as<T>(),
                     (const int32_t*)ctx->d_physmap.as<int32_t>(), (const T*)ctx->d_lbuf.as<T>(), k0p);
      }
    }
    // L11 columns of every panel in pivot order (row exchanges of later panels),
    // from the side buffer into the front
    if (maxp > 0) {
      auto wp = level_sum([&](const NodeInfo& ni, double& by, double& fl) { by += 2.0 * ni.p * ni.p * sz; });
      timed(tm, HF_K_PERMUTE_L11, wp.first, 0.0, s, [&] {
        dim3 g1(cdiv(maxp, NBP), (unsigned)nl);
        k_l11_gather<T><<<g1, 256, 0, s>>>(lnodes, nodes, st, ctx->d_piv.as<int32_t>(), ctx->d_snap.as<int32_t>(),
                                           ctx->d_lbuf.as<T>(), front);
        dim3 g2(cdiv(maxp, 64), cdiv(maxp, 64), (unsigned)nl);
        k_l11_back<T><<<g2, 256, 0, s>>>(lnodes, nodes, st, ctx->d_dval.as<T>(), front);
      });
    }
    // inverses of the 64x64 diagonal blocks of the level's L11 (TRSM and sweeps)
    if (maxp > 0) {
      dim3 gi(cdiv(maxp, 64), (unsigned)nl);
      launch_timed(tm, HF_K_OTHER, 0.0, 0.0, s, k_inv_diag<T>, gi, dim3(256), lnodes, nodes, (const NodeState*)st,
                   (const T*)front, (const int64_t*)ctx->d_linv_off.as<int64_t>(), ctx->d_linv.as<T>());
      // and of the sweep step blocks, built from them
      step_inverses<T>(ctx, l, s);
    }
    // F21, F22
    const int maxb = ctx->level_maxb[l];
    if (maxb > 0) {
      auto w3 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        const double b = ni.b, p = ni.p;
        by += (2.0 * b * p + 0.5 * p * p) * sz;  // F21 read, L21 written, L11 read
        fl += b * p * p;
      });
      auto wg = level_sum([&](const NodeInfo& ni, double& by, double& fl) { by += 2.0 * ni.b * ni.p * sz; });
      dim3 gg(cdiv(maxp, 64), cdiv(maxb, 64), (unsigned)nl);
      launch_timed(tm, HF_K_GATHER_BORDER, wg.first, 0.0, s, k_gather_border<T>, gg, dim3(256), lnodes, nodes,
                   (const NodeState*)st, (const int32_t*)ctx->d_piv.as<int32_t>(), front);
      // windows of one sweep step: the solved columns' contribution to a window
      // is one GEMM over the whole border, the window itself one product with
      // the inverse of its diagonal block
      constexpr int TW = HF_SWEEP_STEP;
      timed(tm, HF_K_TRSM, w3.first, w3.second, s, [&] {
        // stages of k: long over few workgroups, short (several per CU) over many
        constexpr int KBN = SweepStage<T>::value, KBW = SweepStage<T>::value / 4;
        for (int j0 = 0; j0 < maxp; j0 += TW) {
          dim3 gw(cdiv(maxb, 64), TW / 64, (unsigned)nl);
          const bool wide = (int64_t)gw.x * gw.y * gw.z >= 1024;
          if (j0 > 0) {
            auto kg = wide ? k_trsm_gemm<T, KBW> : k_trsm_gemm<T, KBN>;
            kg<<<gw, 256, 0, s>>>(lnodes, nodes, st, front, ctx->d_dval.as<T>(), j0);
          }
          auto ka = wide ? k_trsm_apply<T, KBW> : k_trsm_apply<T, KBN>;
          ka<<<gw, 256, 0, s>>>(lnodes, nodes, st, front, ctx->d_dval.as<T>(), ctx->d_linv2_off.as<int64_t>(),
                                ctx->d_linv2.as<T>(), j0);
        }
      });
      // borders of 512 rows and more: 128 x 128 tiles (FP32 / FP64 products)
      const bool big = maxb >= 512 && h16 == 0 && sizeof(T) == 4;
      const int nt = big ? (maxb + 127) / 128 : (maxb + 63) / 64;
      dim3 g2((unsigned)(nt * (nt + 1) / 2), (unsigned)nl);
      auto w4 = level_sum([&](const NodeInfo& ni, double& by, double& fl) {
        const double b = ni.b, p = ni.p;
        by += (b * p + b * b) * sz;
        fl += b * b * p;
      });
      constexpr int S1 = sizeof(T) == 4 ? 1 : 0, S2 = sizeof(T) == 4 ? 2 : 0;
      launch_timed(tm, HF_K_SYRK, w4.first, w4.second, s,
                   big ? k_syrk128<T> : h16 == 1 ? k_syrk<T, S1> : h16 == 2 ? k_syrk<T, S2> : k_syrk<T>, g2,
                   dim3(256), lnodes, nodes,
                   (const NodeState*)st, front, (const T*)ctx->d_dval.as<T>());
    }
    HF_HIP(hipGetLastError());
  }
  node_inverses<T>(ctx, s);
  ctx->d_ipos.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
  if (ctx->n_nodes > 0) {
    k_mark_l2<<<ctx->n_nodes, 256, 0, s>>>(ctx->n_nodes, nodes, st, ctx->d_piv.as<int32_t>(),
                                           ctx->d_isl2.as<uint8_t>());
    k_inverse_pivots<<<ctx->n_nodes, 256, 0, s>>>(ctx->n_nodes, nodes, ctx->d_piv.as<int32_t>(),
                                                  ctx->d_ipos.as<int32_t>());
  }
  HF_HIP(hipGetLastError());
}

template void step1<float>(hf_ctx*, const double*, hipStream_t);
template void step1<double>(hf_ctx*, const double*, hipStream_t);

}  // namespace hf
