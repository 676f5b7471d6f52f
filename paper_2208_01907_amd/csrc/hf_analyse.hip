// Symbolic analysis on the host (nested-dissection tree of Sec. 2.2).
//
// Input validation, the pattern in elimination order, the border of every tree
// node (the ancestor indices coupled to its subtree), the map from each node's
// border to positions in its parent's front (for the extend-add), the map from
// matrix entries to front positions (for assembly), and the level schedule:
// nodes grouped by height so that each level only depends on finished levels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "hf_internal.h"

namespace hf {

int validate_csr(int64_t n, const int64_t* indptr, const int32_t* indices) {
  if (indptr[0] != 0) return HF_ERR_PATTERN;
  for (int64_t i = 0; i < n; ++i) {
    if (indptr[i + 1] < indptr[i]) return HF_ERR_PATTERN;
    bool diag = false;
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
      const int32_t c = indices[e];
      if (c < 0 || c >= n) return HF_ERR_PATTERN;
      if (e > indptr[i] && indices[e - 1] >= c) return HF_ERR_PATTERN;  // sorted, unique
      if (c == i) diag = true;
    }
    if (!diag) return HF_ERR_PATTERN;
  }
  // structural symmetry: every (i, c) has (c, i)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
      const int32_t c = indices[e];
      const int32_t* b = indices + indptr[c];
      const int32_t* en = indices + indptr[c + 1];
      const int32_t* it = std::lower_bound(b, en, (int32_t)i);
      if (it == en || *it != i) return HF_ERR_PATTERN;
    }
  }
  return HF_OK;
}


int analyse_impl(int64_t n, const int64_t* indptr_h, const int32_t* indices_h, const int32_t* perm_h,
                 int32_t n_nodes, const int32_t* node_ptr_h, const int32_t* parent_h,
                 const hf_options* opt, hf_ctx** out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out || n < 0) return HF_ERR_ARG;
  if (n > 0 && (!indptr_h || !indices_h)) return HF_ERR_ARG;
  if (n >= (int64_t)1 << 31) return HF_ERR_ARG;
  bool single = (node_ptr_h == nullptr && parent_h == nullptr);
  if (!single && (!node_ptr_h || !parent_h || n_nodes < 1)) return HF_ERR_ARG;
  hf_options o;
  hf_default_options(&o);
  if (opt) o = *opt;
  if (o.nd_leaf_max < 1) return HF_ERR_ARG;
  // neither an ordering nor a tree: nested dissection of the pattern (Sec. 2.2)
  std::vector<int32_t> nd_perm, nd_ptr, nd_parent;
  if (single && !perm_h && n > o.nd_leaf_max) {
    try {
      nd_perm.resize((size_t)n);
      nd_ptr.resize((size_t)n + 1);
      nd_parent.resize((size_t)n);
    } catch (const std::bad_alloc&) {
      return HF_ERR_OOM;
    }
    int32_t nn = 0;
    const int rc = order_impl(n, indptr_h, indices_h, o.nd_leaf_max, nd_perm.data(), &nn, nd_ptr.data(),
                              nd_parent.data());
    if (rc) return rc;
    perm_h = nd_perm.data();
    node_ptr_h = nd_ptr.data();
    parent_h = nd_parent.data();
    n_nodes = nn;
    single = false;
  }
  if (!(o.tau >= 0.0) || !std::isfinite(o.tau)) return HF_ERR_ARG;
  if (o.low_precision != HF_PREC_FP16 && o.low_precision != HF_PREC_FP16_PAIR && o.low_precision != HF_PREC_FP32 &&
      o.low_precision != HF_PREC_FP64)
    return HF_ERR_ARG;
  if (o.n_enlarge < 0 || o.gcr_block < 0 || o.gcr_block > 64 || o.gcr_maxit < 1 || !(o.gcr_tol > 0) ||
      !(o.ker_tol >= 0) || o.refine_steps < 0 || o.refine_steps > 8 || !(o.refine_tol > 0) ||
      o.sweep_front_min < 0 || o.sweep_wide_min < 1 ||
      o.sweep_node_inverse < 0 || o.sweep_node_inverse > 2)
    return HF_ERR_ARG;
  if (n > 0) {
    int rc = validate_csr(n, indptr_h, indices_h);
    if (rc) return rc;
  }
  hf_ctx* ctx = new (std::nothrow) hf_ctx();
  if (!ctx) return HF_ERR_OOM;
  try {
    ctx->opt = o;
    ctx->n = n;
    ctx->nnz = n > 0 ? indptr_h[n] : 0;
    const int64_t nnz = ctx->nnz;
    ctx->indptr.assign(indptr_h, indptr_h + n + 1);
    ctx->indices.assign(indices_h, indices_h + nnz);
    // permutation
    ctx->perm.resize(n);
    ctx->iperm.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      const int32_t o2 = perm_h ? perm_h[k] : (int32_t)k;
      if (o2 < 0 || o2 >= n || ctx->iperm[o2] >= 0) { delete ctx; return HF_ERR_ARG; }
      ctx->perm[k] = o2;
      ctx->iperm[o2] = (int32_t)k;
    }
    // tree
    if (single) {
      n_nodes = 1;
      ctx->node_ptr = {0, (int32_t)n};
      ctx->parent = {-1};
    } else {
      ctx->node_ptr.assign(node_ptr_h, node_ptr_h + n_nodes + 1);
      ctx->parent.assign(parent_h, parent_h + n_nodes);
    }
    ctx->n_nodes = n_nodes;
    auto& np = ctx->node_ptr;
    auto& par = ctx->parent;
    if (np[0] != 0 || np[n_nodes] != n) { delete ctx; return HF_ERR_ARG; }
    for (int32_t j = 0; j < n_nodes; ++j) {
      if (np[j + 1] < np[j]) { delete ctx; return HF_ERR_ARG; }
      if (par[j] != -1 && (par[j] <= j || par[j] >= n_nodes)) { delete ctx; return HF_ERR_ARG; }
      if (np[j + 1] - np[j] > 4096) { delete ctx; return HF_ERR_NOT_IMPLEMENTED; }
    }
    // children, subtree ranges (postorder contiguity)
    std::vector<int32_t> nch(n_nodes, 0), first(n_nodes), nsub(n_nodes, 1);
    for (int32_t j = 0; j < n_nodes; ++j) first[j] = j;
    for (int32_t j = 0; j < n_nodes; ++j) {
      if (par[j] >= 0) {
        nch[par[j]]++;
        first[par[j]] = std::min(first[par[j]], first[j]);
        nsub[par[j]] += nsub[j];
      }
    }
    for (int32_t j = 0; j < n_nodes; ++j)
      if (nsub[j] != j - first[j] + 1) { delete ctx; return HF_ERR_ARG; }
    std::vector<int32_t> cptr(n_nodes + 1, 0), fill(n_nodes, 0);
    for (int32_t j = 0; j < n_nodes; ++j) cptr[j + 1] = cptr[j] + nch[j];
    ctx->child_list.assign(std::max<int32_t>(cptr[n_nodes], 1), 0);
    for (int32_t j = 0; j < n_nodes; ++j)
      if (par[j] >= 0) ctx->child_list[cptr[par[j]] + fill[par[j]]++] = j;
    std::vector<int32_t> node_of(n);
    for (int32_t j = 0; j < n_nodes; ++j)
      for (int32_t g = np[j]; g < np[j + 1]; ++g) node_of[g] = j;

    // pattern in elimination order
    std::vector<int64_t> pindptr(n + 1, 0);
    for (int64_t g = 0; g < n; ++g) {
      const int32_t o2 = ctx->perm[g];
      pindptr[g + 1] = pindptr[g] + (indptr_h[o2 + 1] - indptr_h[o2]);
    }
    std::vector<int32_t> pindices(nnz);
    std::vector<int64_t> psrc(nnz);
    std::vector<int32_t> diagpos(n);
    {
      std::vector<std::pair<int32_t, int64_t>> row;
      for (int64_t g = 0; g < n; ++g) {
        const int32_t o2 = ctx->perm[g];
        row.clear();
        for (int64_t e = indptr_h[o2]; e < indptr_h[o2 + 1]; ++e)
          row.emplace_back(ctx->iperm[indices_h[e]], e);
        std::sort(row.begin(), row.end());
        int64_t w = pindptr[g];
        for (auto& pr : row) {
          if (pr.first == g) diagpos[g] = (int32_t)(w - pindptr[g]);
          pindices[w] = pr.first;
          psrc[w] = pr.second;
          ++w;
        }
      }
    }
    // validate couplings against the tree and build the borders (postorder)
    ctx->border_ptr.assign(n_nodes + 1, 0);
    std::vector<std::vector<int32_t>> borders(n_nodes);
    std::vector<int32_t> mark(n, -1);
    for (int32_t j = 0; j < n_nodes; ++j) {
      const int32_t s = np[j], e = np[j + 1];
      const int32_t sub_start = np[first[j]];
      std::vector<int32_t>& bj = borders[j];
      for (int32_t g = s; g < e; ++g) {
        for (int64_t q = pindptr[g]; q < pindptr[g + 1]; ++q) {
          const int32_t c = pindices[q];
          if (c < sub_start) { delete ctx; return HF_ERR_PATTERN; }
          if (c >= e) {
            const int32_t o2 = node_of[c];
            if (first[o2] > j) { delete ctx; return HF_ERR_PATTERN; }  // not an ancestor
            if (mark[c] != j) { mark[c] = j; bj.push_back(c); }
          }
        }
      }
      for (int32_t ci = cptr[j]; ci < cptr[j + 1]; ++ci) {
        for (int32_t c : borders[ctx->child_list[ci]]) {
          if (c >= e && mark[c] != j) { mark[c] = j; bj.push_back(c); }
        }
      }
      std::sort(bj.begin(), bj.end());
      ctx->border_ptr[j + 1] = ctx->border_ptr[j] + (int64_t)bj.size();
    }
    if (ctx->border_ptr[n_nodes] >= ((int64_t)1 << 31)) { delete ctx; return HF_ERR_NOT_IMPLEMENTED; }
    ctx->border.resize(ctx->border_ptr[n_nodes]);
    for (int32_t j = 0; j < n_nodes; ++j)
      std::copy(borders[j].begin(), borders[j].end(), ctx->border.begin() + ctx->border_ptr[j]);

    // node records, arena offsets, cost model
    ctx->nodes.resize(n_nodes);
    int64_t off = 0, roff = 0, soff = 0, loff = 0;
    ctx->flops_sym = 0.0;
    ctx->factor_entries = 0;
    for (int32_t j = 0; j < n_nodes; ++j) {
      NodeInfo& ni = ctx->nodes[j];
      ni.start = np[j];
      ni.p = np[j + 1] - np[j];
      ni.b = (int32_t)(ctx->border_ptr[j + 1] - ctx->border_ptr[j]);
      ni.f = ni.p + ni.b;
      if ((int64_t)ni.f * ni.f >= ((int64_t)1 << 31)) { delete ctx; return HF_ERR_NOT_IMPLEMENTED; }  // 32-bit front offsets
      ni.parent = par[j];
      ni.child_begin = cptr[j];
      ni.child_end = cptr[j + 1];
      ni.border_off = (int32_t)ctx->border_ptr[j];
      ni.front_off = off;
      ni.rhs_off = roff;
      ni.snap_off = soff;
      ni.lbuf_ld = (ni.p + 3) & ~3;
      ni.lbuf_off = loff;
      loff += (int64_t)ni.p * ni.lbuf_ld;
      off += (int64_t)ni.f * ni.f;
      roff += ni.f;
      soff += (int64_t)((ni.p + 7) / 8) * ni.p;  // panels of at least 8 pivots
      ctx->max_front = std::max(ctx->max_front, ni.f);
      ctx->max_p = std::max(ctx->max_p, ni.p);
      const double p = ni.p, f = ni.f;
      // lower-triangle rank-1 updates: sum_{i<p} (f-i-1)(f-i) flops, plus divisions
      ctx->flops_sym += p * f * f - p * p * f + p * p * p / 3.0;
      ctx->factor_entries += (int64_t)ni.f * ni.p - (int64_t)ni.p * (ni.p - 1) / 2;
    }
    ctx->front_elems = off;
    ctx->rhs_rows = roff;
    ctx->snap_elems = soff;
    ctx->lbuf_elems = loff;
    // border -> parent-front positions
    ctx->relmap.assign(std::max<int64_t>(ctx->border.size(), 1), 0);
    for (int32_t j = 0; j < n_nodes; ++j) {
      const int32_t P = par[j];
      for (int64_t q = ctx->border_ptr[j]; q < ctx->border_ptr[j + 1]; ++q) {
        const int32_t x = ctx->border[q];
        int32_t pos;
        if (P < 0) { delete ctx; return HF_ERR_PATTERN; }  // a root cannot have a border
        if (x >= np[P] && x < np[P + 1]) {
          pos = x - np[P];
        } else {
          const int32_t* b = ctx->border.data() + ctx->border_ptr[P];
          const int32_t* en = ctx->border.data() + ctx->border_ptr[P + 1];
          const int32_t* it = std::lower_bound(b, en, x);
          if (it == en || *it != x) { delete ctx; return HF_ERR_PATTERN; }
          pos = ctx->nodes[P].p + (int32_t)(it - b);
        }
        ctx->relmap[q] = pos;
      }
    }
    // entry -> front position (lower triangle; entries with col < row are assembled
    // from their mirror image)
    std::vector<int64_t> asmmap(nnz, -1);
    for (int64_t g = 0; g < n; ++g) {
      const int32_t j = node_of[g];
      const NodeInfo& ni = ctx->nodes[j];
      const int32_t colpos = (int32_t)g - ni.start;
      for (int64_t q = pindptr[g]; q < pindptr[g + 1]; ++q) {
        const int32_t c = pindices[q];
        if (c < g) continue;
        int32_t rowpos;
        if (c < ni.start + ni.p) {
          rowpos = c - ni.start;
        } else {
          const int32_t* b = ctx->border.data() + ctx->border_ptr[j];
          const int32_t* en = ctx->border.data() + ctx->border_ptr[j + 1];
          const int32_t* it = std::lower_bound(b, en, c);
          rowpos = ni.p + (int32_t)(it - b);
        }
        asmmap[q] = ni.front_off + (int64_t)colpos * ni.f + rowpos;
      }
    }
    // height levels
    std::vector<int32_t> h(n_nodes, 0);
    int32_t H = 0;
    for (int32_t j = 0; j < n_nodes; ++j) {
      if (par[j] >= 0) h[par[j]] = std::max(h[par[j]], h[j] + 1);
      H = std::max(H, h[j]);
    }
    const int32_t nlev = n_nodes > 0 ? H + 1 : 0;
    ctx->level_ptr.assign(nlev + 1, 0);
    for (int32_t j = 0; j < n_nodes; ++j) ctx->level_ptr[h[j] + 1]++;
    for (int32_t l = 0; l < nlev; ++l) ctx->level_ptr[l + 1] += ctx->level_ptr[l];
    ctx->level_nodes.assign(std::max(n_nodes, 1), 0);
    {
      std::vector<int32_t> lf(nlev, 0);
      for (int32_t j = 0; j < n_nodes; ++j) ctx->level_nodes[ctx->level_ptr[h[j]] + lf[h[j]]++] = j;
    }
    ctx->level_maxp.assign(nlev, 0);
    ctx->level_maxf.assign(nlev, 0);
    ctx->level_maxb.assign(nlev, 0);
    ctx->level_maxc.assign(nlev, 0);
    for (int32_t l = 0; l < nlev; ++l) {
      for (int32_t q = ctx->level_ptr[l]; q < ctx->level_ptr[l + 1]; ++q) {
        const NodeInfo& ni = ctx->nodes[ctx->level_nodes[q]];
        ctx->level_maxp[l] = std::max(ctx->level_maxp[l], ni.p);
        ctx->level_maxf[l] = std::max(ctx->level_maxf[l], ni.f);
        ctx->level_maxb[l] = std::max(ctx->level_maxb[l], ni.b);
        ctx->level_maxc[l] = std::max(ctx->level_maxc[l], ni.child_end - ni.child_begin);
      }
    }

    // extend-add launches: per level, one per child rank, children with a border
    for (int32_t l = 0; l < nlev; ++l) {
      for (int32_t rank = 0; rank < ctx->level_maxc[l]; ++rank) {
        EaLaunch el{l, rank, (int32_t)ctx->ea_items.size(), 0, 0};
        for (int32_t q = ctx->level_ptr[l]; q < ctx->level_ptr[l + 1]; ++q) {
          const NodeInfo& ni = ctx->nodes[ctx->level_nodes[q]];
          if (ni.child_begin + rank < ni.child_end) {
            const int32_t c = ctx->child_list[ni.child_begin + rank];
            if (ctx->nodes[c].b > 0) {
              ctx->ea_items.push_back(c);
              el.count++;
              el.maxb = std::max(el.maxb, ctx->nodes[c].b);
            }
          }
        }
        if (el.count) ctx->ea_launch.push_back(el);
      }
    }
    // forward-sweep gather: for every front row (slot rhs_off + assembly position),
    // the children's border rows added into it, children in rank order
    {
      std::vector<int64_t> cnt((size_t)ctx->rhs_rows + 1, 0);
      for (int32_t c = 0; c < n_nodes; ++c) {
        const NodeInfo& cn = ctx->nodes[c];
        if (cn.parent < 0) continue;
        const NodeInfo& pn = ctx->nodes[cn.parent];
        for (int32_t r = 0; r < cn.b; ++r) cnt[pn.rhs_off + ctx->relmap[cn.border_off + r] + 1]++;
      }
      for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
      ctx->gat_ptr = cnt;
      ctx->gat_src.assign(std::max<int64_t>(cnt.back(), 1), 0);
      std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
      for (int32_t j = 0; j < n_nodes; ++j) {
        const NodeInfo& pn = ctx->nodes[j];
        for (int32_t q = pn.child_begin; q < pn.child_end; ++q) {  // rank order
          const int32_t c = ctx->child_list[q];
          const NodeInfo& cn = ctx->nodes[c];
          for (int32_t r = 0; r < cn.b; ++r)
            ctx->gat_src[fill[pn.rhs_off + ctx->relmap[cn.border_off + r]]++] = cn.rhs_off + cn.p + r;
        }
      }
    }
    // 64x64 diagonal blocks of every node (inverted after each factorization)
    ctx->blk_first.assign(n_nodes + 1, 0);
    ctx->linv_off.assign(std::max(n_nodes, 1), 0);
    for (int32_t j = 0; j < n_nodes; ++j) {
      const int32_t nb = (ctx->nodes[j].p + 63) / 64;
      ctx->linv_off[j] = (int64_t)ctx->blk_first[j] * 64 * 64;
      ctx->blk_first[j + 1] = ctx->blk_first[j] + nb;
      for (int32_t q = 0; q < nb; ++q) ctx->blk_node.push_back(j);
    }
    ctx->linv_elems = (int64_t)ctx->blk_first[n_nodes] * 64 * 64;
    // step blocks of the triangular sweeps (their inverses drive them)
    // numbered level by level, so that the steps of one level are contiguous (their
    // inverses are formed with the level, before its TRSM)
    ctx->stp_first.assign(n_nodes + 1, 0);
    ctx->linv2_off.assign(std::max(n_nodes, 1), 0);
    ctx->lvl_step_ptr.assign(nlev + 1, 0);
    int32_t nsteps = 0;
    for (int32_t l = 0; l < nlev; ++l) {
      for (int32_t q = ctx->level_ptr[l]; q < ctx->level_ptr[l + 1]; ++q) {
        const int32_t j = ctx->level_nodes[q];
        const int32_t nb = (ctx->nodes[j].p + HF_SWEEP_STEP - 1) / HF_SWEEP_STEP;
        ctx->stp_first[j] = nsteps;
        ctx->linv2_off[j] = (int64_t)nsteps * HF_SWEEP_STEP * HF_SWEEP_STEP;
        for (int32_t t = 0; t < nb; ++t) ctx->stp_node.push_back(j);
        nsteps += nb;
      }
      ctx->lvl_step_ptr[l + 1] = nsteps;
    }
    ctx->stp_first[n_nodes] = nsteps;
    ctx->linv2_elems = (int64_t)nsteps * HF_SWEEP_STEP * HF_SWEEP_STEP;
    // node inverses: every node of more than one step, leading dimension p
    // rounded up to 64; the merges of recursive doubling pair blocks of TB << t
    // columns [a0, a0 + s) and [a0 + s, a0 + 2s) while the second one starts
    // inside the node (the pivot count can only trim them)
    ctx->ninv_off.assign(std::max(n_nodes, 1), -1);
    ctx->ninv_ld.assign(std::max(n_nodes, 1), 0);
    ctx->ninv_elems = 0;
    ctx->ninv_lvl.assign(1, 0);
    if (o.sweep_node_inverse) {
      for (int32_t j = 0; j < n_nodes; ++j) {
        const int32_t p = ctx->nodes[j].p;
        if (p <= HF_SWEEP_STEP) continue;
        const int32_t ld = (p + 63) / 64 * 64;
        ctx->ninv_off[j] = ctx->ninv_elems;
        ctx->ninv_ld[j] = ld;
        ctx->ninv_elems += (int64_t)ld * ld;
        for (int32_t c = 0; c < p; ++c) {  // one sign sum per column
          ctx->ninv_cnode.push_back(j);
          ctx->ninv_ccol.push_back(c);
        }
        for (int32_t t = ctx->stp_first[j]; t < ctx->stp_first[j] + (p + HF_SWEEP_STEP - 1) / HF_SWEEP_STEP; ++t)
          ctx->ninv_copy.push_back(t);
      }
      for (int64_t sb = HF_SWEEP_STEP; sb < ctx->max_p; sb *= 2) {
        for (int32_t j = 0; j < n_nodes; ++j) {
          if (ctx->ninv_off[j] < 0) continue;
          for (int64_t a0 = 0; a0 + sb < ctx->nodes[j].p; a0 += 2 * sb) {
            ctx->ninv_jnode.push_back(j);
            ctx->ninv_ja0.push_back((int32_t)a0);
          }
        }
        ctx->ninv_lvl.push_back((int32_t)ctx->ninv_jnode.size());
      }
    }
    // device copies of the pattern
    hipStream_t s = nullptr;
    upload(ctx->d_pindptr, pindptr, s);
    upload(ctx->d_pindices, pindices, s);
    upload(ctx->d_psrc, psrc, s);
    upload(ctx->d_diagpos, diagpos, s);
    upload(ctx->d_asm, asmmap, s);
    upload(ctx->d_perm, ctx->perm, s);
    upload(ctx->d_iperm, ctx->iperm, s);
    upload(ctx->d_nodes, ctx->nodes, s);
    upload(ctx->d_border, ctx->border, s);
    upload(ctx->d_relmap, ctx->relmap, s);
    upload(ctx->d_level_nodes, ctx->level_nodes, s);
    upload(ctx->d_child_list, ctx->child_list, s);
    upload(ctx->d_ea_items, ctx->ea_items, s);
    upload(ctx->d_gat_ptr, ctx->gat_ptr, s);
    upload(ctx->d_gat_src, ctx->gat_src, s);
    upload(ctx->d_blk_node, ctx->blk_node, s);
    upload(ctx->d_blk_first, ctx->blk_first, s);
    upload(ctx->d_linv_off, ctx->linv_off, s);
    upload(ctx->d_stp_node, ctx->stp_node, s);
    upload(ctx->d_stp_first, ctx->stp_first, s);
    upload(ctx->d_linv2_off, ctx->linv2_off, s);
    upload(ctx->d_ninv_off, ctx->ninv_off, s);
    upload(ctx->d_ninv_ld, ctx->ninv_ld, s);
    upload(ctx->d_ninv_copy, ctx->ninv_copy, s);
    upload(ctx->d_ninv_jnode, ctx->ninv_jnode, s);
    upload(ctx->d_ninv_ja0, ctx->ninv_ja0, s);
    {
      // the root of every node's tree (nodes are numbered children first)
      std::vector<int32_t> rootof(std::max(n_nodes, 1), 0);
      for (int32_t j = n_nodes - 1; j >= 0; --j) rootof[j] = par[j] >= 0 ? rootof[par[j]] : j;
      // independent trees (no root has a border): the sweeps and block GCR may
      // leave out the trees a right-hand side does not touch
      ctx->n_roots = 0;
      bool indep = true;
      for (int32_t j = 0; j < n_nodes; ++j)
        if (par[j] < 0) {
          ++ctx->n_roots;
          indep = indep && ctx->nodes[j].b == 0;
        }
      if (!indep) ctx->n_roots = 1;
      // the rows spanned by every tree (block GCR runs on the trees its
      // right-hand sides touch), and the tree of every row
      ctx->tree_lo.assign(std::max(n_nodes, 1), INT64_MAX);
      ctx->tree_hi.assign(std::max(n_nodes, 1), 0);
      ctx->row_tree.assign((size_t)n, 0);
      for (int32_t j = 0; j < n_nodes; ++j) {
        const int32_t r = rootof[j];
        const NodeInfo& ni = ctx->nodes[j];
        ctx->tree_lo[r] = std::min<int64_t>(ctx->tree_lo[r], ni.start);
        ctx->tree_hi[r] = std::max<int64_t>(ctx->tree_hi[r], (int64_t)ni.start + ni.p);
        for (int32_t g = ni.start; g < ni.start + ni.p; ++g) ctx->row_tree[g] = r;
      }
      upload(ctx->d_rootof, rootof, s);
    }
    upload(ctx->d_ninv_cnode, ctx->ninv_cnode, s);
    upload(ctx->d_ninv_ccol, ctx->ninv_ccol, s);
    HF_HIP(hipStreamSynchronize(s));
    ctx->state = 1;
  } catch (const HipError&) {
    delete ctx;
    return HF_ERR_HIP;
  } catch (const Status& st) {
    delete ctx;
    return st.code;
  } catch (const std::bad_alloc&) {
    delete ctx;
    return HF_ERR_OOM;
  }
  ctx->t_analyse =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = ctx;
  return HF_OK;
}

}  // namespace hf
