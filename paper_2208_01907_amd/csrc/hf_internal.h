// Internal declarations of the hybrid factorization library (host side).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hf.h"

namespace hf {

// columns of L11 per step of the triangular sweeps (explicit inverse per step)
constexpr int HF_SWEEP_STEP = 512;


struct HipError {
  hipError_t err;
};

#define HF_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) throw ::hf::HipError{e_};    \
  } while (0)

struct Status {
  int code;
};

// Device buffer owned by the context.
struct DBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  void alloc(size_t nbytes) {
    if (nbytes <= bytes && ptr) return;
    release();
    if (nbytes == 0) nbytes = 16;
    if (hipMalloc(&ptr, nbytes) != hipSuccess) {
      ptr = nullptr;
      throw Status{HF_ERR_OOM};
    }
    bytes = nbytes;
  }
  template <class T>
  T* as() const { return static_cast<T*>(ptr); }
};

template <class T>
void upload(DBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) HF_HIP(hipMemcpyAsync(d.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Per-node record uploaded to the device (all sizes in elements).
struct NodeInfo {
  int64_t front_off;  // offset of the front in the arena
  int64_t rhs_off;    // offset (rows) of the node's block in the solve arena
  int64_t snap_off;   // offset of the node's per-panel position -> index snapshots
  int64_t lbuf_off;   // offset of the node's panel columns of L (p columns, leading dimension lbuf_ld)
  int32_t start;      // first position of the node in elimination order
  int32_t p;          // pivot candidates
  int32_t b;          // border size
  int32_t f;          // p + b
  int32_t parent;
  int32_t child_begin;  // into child_list
  int32_t child_end;
  int32_t border_off;   // into border / relmap (int32 is enough: < 2^31 entries)
  int32_t lbuf_ld;      // p rounded up to a multiple of 4
};

// Mutable per-node factorization state on the device.
struct NodeState {
  int32_t npiv;   // accepted pivots so far
  int32_t done;   // 1 when the node's pivot block is finished
  double dprev;   // last accepted pivot (ratio reference)
  double dstop;   // diagonal value of the candidate that stopped the node (NaN: none did)
};

// One extend-add launch: the children of rank `rank` of the nodes of a level.
struct EaLaunch {
  int32_t level, rank, off, count, maxb;
};

struct BgcrWork;

// Event timing of instrumented launches (see hf_timing_enable).
struct KTimer {
  bool on = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  double ms[HF_K_NCLASS] = {};
  int64_t n[HF_K_NCLASS] = {};
  double bytes[HF_K_NCLASS] = {};
  double flops[HF_K_NCLASS] = {};
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) throw HipError{hipErrorOutOfMemory};
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    for (int c = 0; c < HF_K_NCLASS; ++c) { ms[c] = 0; n[c] = 0; bytes[c] = 0; flops[c] = 0; }
    recs.clear();
    used = 0;
  }
  // after the stream is synchronized
  void flush() {
    for (auto& r : recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) ms[r.cls] += t;
      n[r.cls] += 1;
      bytes[r.cls] += r.bytes;
      flops[r.cls] += r.flops;
    }
    recs.clear();
    used = 0;
  }
  ~KTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Launch wrapper: brackets `launch` with events when timing is on.
template <class F>
inline void timed(KTimer& tm, int cls, double bytes, double flops, hipStream_t s, F&& launch) {
  if (!tm.on) {
    launch();
    return;
  }
  hipEvent_t a = tm.next(), b = tm.next();
  HF_HIP(hipEventRecord(a, s));
  launch();
  HF_HIP(hipEventRecord(b, s));
  tm.recs.push_back({cls, a, b, bytes, flops});
}

// Single-kernel launch; with timing on, the events take the start and end of
// the kernel's own execution (dispatch profiling), not the stream positions
// around it, so the per-kernel times exclude launch gaps.
template <class K, class... A>
inline void launch_timed(KTimer& tm, int cls, double bytes, double flops, hipStream_t s, K kernel, dim3 grid,
                         dim3 block, A... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm.on) {
    a = tm.next();
    b = tm.next();
    tm.recs.push_back({cls, a, b, bytes, flops});
  }
  hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, args...);
}

}  // namespace hf

struct hf_ctx {
  hf_options opt{};
  int state = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> indptr;
  std::vector<int32_t> indices;
  std::vector<int32_t> perm, iperm;
  int32_t n_nodes = 0;
  std::vector<int32_t> node_ptr, parent;
  // symbolic
  std::vector<int64_t> border_ptr;
  std::vector<int32_t> border, relmap;
  std::vector<hf::NodeInfo> nodes;
  std::vector<int32_t> child_list;
  std::vector<int32_t> level_ptr, level_nodes;  // height levels, leaves first
  std::vector<int32_t> level_maxp, level_maxf, level_maxb, level_maxc;
  std::vector<hf::EaLaunch> ea_launch;
  std::vector<int32_t> blk_node, blk_first;  // 64-row diagonal blocks of every L11
  std::vector<int64_t> linv_off;
  int64_t linv_elems = 0;
  std::vector<int32_t> stp_node, stp_first;  // sweep steps of every L11 (numbered level by level)
  std::vector<int32_t> lvl_step_ptr;         // steps of level l: [lvl_step_ptr[l], lvl_step_ptr[l + 1])
  std::vector<int64_t> linv2_off;
  int64_t linv2_elems = 0;
  // explicit inverse of the L11 of every node of more than one sweep step
  // (column-major, leading dimension ninv_ld[j]; ninv_off[j] < 0: none)
  std::vector<int64_t> ninv_off;
  std::vector<int32_t> ninv_ld;
  int64_t ninv_elems = 0;
  std::vector<int32_t> ninv_copy;                  // sweep steps whose inverse is copied in
  std::vector<int32_t> ninv_jnode, ninv_ja0;       // merges: node, first column of the pair
  std::vector<int32_t> ninv_lvl;                   // merges of block size TB << t: [ninv_lvl[t], ninv_lvl[t + 1])
  std::vector<int32_t> ninv_cnode, ninv_ccol;      // every column of every node inverse: node, column
  std::vector<uint8_t> level_one_pass;             // per level: the sweeps take the node inverses
  std::vector<int32_t> ea_items;
  std::vector<int64_t> gat_ptr, gat_src;  // per front-row slot: the child slab rows added into it
  int64_t front_elems = 0, rhs_rows = 0, snap_elems = 0, lbuf_elems = 0;
  int32_t max_front = 0, max_p = 0;
  double flops_sym = 0.0, flops_done = 0.0;
  int64_t factor_entries = 0;
  // device: pattern
  hf::DBuf d_pindptr, d_pindices, d_psrc, d_diagpos, d_asm;
  hf::DBuf d_orow, d_ocol;         // caller's pattern, one (row, column) per entry (adjoint)
  hf::DBuf d_perm, d_iperm, d_nodes, d_border, d_relmap, d_level_nodes, d_child_list, d_ea_items;
  hf::DBuf d_gat_ptr, d_gat_src;
  // device: numeric
  hf::DBuf d_q, d_kval;            // scaling, scaled FP64 values (elimination order)
  hf::DBuf d_kbar;                 // the caller's FP64 values in elimination order
  hf::DBuf d_front;                // front arena (T = float or double)
  hf::DBuf d_state, d_piv, d_dval; // NodeState[n_nodes], piv_order[n], D[n] (T)
  hf::DBuf d_ipos;                 // position of each index in its node's pivot order
  hf::DBuf d_snap;                 // per panel: index at every position of the node when it ended
  hf::DBuf d_physmap;              // per position: storage index after the last panel
  hf::DBuf d_lbuf;                 // per node: the panels' L columns, rows in the order of their panel
  hf::DBuf d_linv, d_linv_off, d_blk_node, d_blk_first;  // inverses of 64x64 diagonal blocks
  hf::DBuf d_linv2, d_linv2_off, d_stp_node, d_stp_first;  // inverses of the sweep step blocks
  hf::DBuf d_ninv, d_ninv_off, d_ninv_ld, d_ninv_copy, d_ninv_jnode, d_ninv_ja0;  // node inverses
  hf::DBuf d_ninv_cnode, d_ninv_ccol, d_ninv_bad;  // per node: L11 fails the sign test (no node inverse)
  hf::DBuf d_zb_arena;             // second solve arena (step results)
  hf::DBuf d_part;                 // partial products of the backward border step
  hf::DBuf d_live;                 // per node: last preconditioner application with a nonzero forward block
  hf::DBuf d_tree_live;            // per tree root: the same for any front of the tree
  hf::DBuf d_rootof;               // per node: the root of its tree
  int32_t n_roots = 0;             // trees of the forest
  std::vector<int64_t> tree_lo, tree_hi;  // per tree root: rows [lo, hi) its nodes span
  std::vector<int32_t> row_tree;   // per row (elimination order): the root of its tree
  int32_t live_gen = 0;
  hf::DBuf d_isl2, d_flag;         // uint8 mask [n], error flags
  int32_t factor_prec = 0;         // precision of d_front
  // hard part
  std::vector<int32_t> lambda2;    // elimination-order indices, ascending
  hf::DBuf d_l2;
  int32_t M = 0;
  // X12 in column blocks (row-major n x mb each), S22 and its factorization
  hf::DBuf d_X12, d_S22, d_S22f, d_s22perm, d_s22mag, d_s22info, d_s22slots, d_N2, d_kern, d_ktmp, d_tune;
  std::vector<int64_t> x12_rng;  // rows [lo, hi) of each block of X12 (zero outside)
  hf::DBuf d_x12rng;
  int32_t mb = 0, nblk = 0;
  int32_t kdim = 0;
  double rank_gap = 0.0;
  int32_t rank_candidates = 0;
  // solve-phase scratch
  hf::DBuf d_rhs_arena;            // front RHS arena (T)
  hf::DBuf d_rhs_b, d_y2, d_x2pad; // Algorithm 2 scratch
  hf::DBuf d_adj;                  // adjoint: right-hand sides projected onto the range
  hf::BgcrWork* work = nullptr;
  hf::KTimer timer;
  std::vector<hf::NodeState> hstate;  // node states after the last factorization
  // block-GCR residual histories (max relative recurrence residual over the
  // active columns, after X0 and after every iteration): the Schur-complement
  // runs of the last hf_factorize, then the runs of the last hf_solve
  std::vector<int32_t> hist_ptr{0};
  std::vector<double> hist;
  int32_t hist_factor_runs = 0;
  // statistics
  int32_t gcr_blocks = 0, gcr_iters_max = 0, gcr_iters_total = 0, solve_iters = 0;
  double t_analyse = 0, t_step1 = 0, t_gcr = 0, t_s22 = 0, t_solve = 0;
  ~hf_ctx();
};

namespace hf {
int validate_csr(int64_t n, const int64_t* indptr, const int32_t* indices);
int order_impl(int64_t n, const int64_t* indptr, const int32_t* indices, int32_t leaf_max, int32_t* perm,
               int32_t* n_nodes, int32_t* node_ptr, int32_t* parent);
int analyse_impl(int64_t n, const int64_t* indptr, const int32_t* indices, const int32_t* perm,
                 int32_t n_nodes, const int32_t* node_ptr, const int32_t* parent,
                 const hf_options* opt, hf_ctx** out);
int factorize_impl(hf_ctx* ctx, const double* values, hipStream_t s);
int solve_impl(hf_ctx* ctx, int32_t r, const double* B, int64_t ldb, double* X, int64_t ldx,
               hipStream_t s);
void free_work(hf_ctx* ctx);
int schur_impl(const hf_ctx* ctx, int32_t* m, int32_t* lambda2, double* S, int64_t lds, hipStream_t s);
int kernel_basis_impl(const hf_ctx* ctx, double* N, int64_t ldn, hipStream_t s);
int adjoint_impl(hf_ctx* ctx, int32_t r, const double* X, int64_t ldx, const double* G, int64_t ldg,
                 double* Lam, int64_t ldl, double* GV, hipStream_t s);
int scaling_impl(const hf_ctx* ctx, double* q, hipStream_t s);
int precond_impl(hf_ctx* ctx, int32_t r, const double* R, double* Y, hipStream_t s);
int tune_impl(hf_ctx* ctx, int32_t r, int32_t* front_min, int32_t* wide_min, double* ms, hipStream_t s);
}  // namespace hf
