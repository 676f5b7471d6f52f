// C entry points of include/hf.h.
#include <algorithm>
#include <cmath>
#include <new>

#include "hf_internal.h"

hf_ctx::~hf_ctx() { hf::free_work(this); }

extern "C" {

void hf_default_options(hf_options* opt) {
  if (!opt) return;
  opt->tau = 1e-2;
  opt->low_precision = HF_PREC_FP32;
  opt->first_pivot_unit = 1;
  opt->n_enlarge = 4;
  opt->gcr_block = 0;
  opt->gcr_tol = 1e-15;
  opt->gcr_maxit = 50;
  opt->ker_tol = 1e-10;
  opt->refine_steps = 1;
  opt->refine_tol = 1e-3;
  opt->nd_leaf_max = 512;
  opt->sweep_front_min = 256;
  opt->sweep_wide_min = 256;
  opt->sweep_node_inverse = 1;
}

int hf_analyse(int64_t n, const int64_t* indptr_host, const int32_t* indices_host, const int32_t* perm_host,
               int32_t n_nodes, const int32_t* node_ptr_host, const int32_t* parent_host,
               const hf_options* opt, hf_ctx** out) {
  return hf::analyse_impl(n, indptr_host, indices_host, perm_host, n_nodes, node_ptr_host, parent_host,
                          opt, out);
}

int hf_factorize(hf_ctx* ctx, const double* values_dev, void* stream) {
  if (!ctx) return HF_ERR_ARG;
  return hf::factorize_impl(ctx, values_dev, static_cast<hipStream_t>(stream));
}

int hf_solve(hf_ctx* ctx, int32_t r, const double* B_dev, int64_t ldb, double* X_dev, int64_t ldx,
             void* stream) {
  if (!ctx) return HF_ERR_ARG;
  if (B_dev && X_dev && B_dev == X_dev && r > 0) return HF_ERR_ARG;
  return hf::solve_impl(ctx, r, B_dev, ldb, X_dev, ldx, static_cast<hipStream_t>(stream));
}

int hf_adjoint(hf_ctx* ctx, int32_t r, const double* X_dev, int64_t ldx, const double* G_dev, int64_t ldg,
               double* Lam_dev, int64_t ldl, double* GV_dev, void* stream) {
  if (!ctx) return HF_ERR_ARG;
  if (r > 0 && Lam_dev && (Lam_dev == G_dev || Lam_dev == X_dev)) return HF_ERR_ARG;
  if (r > 0 && GV_dev && (GV_dev == Lam_dev || GV_dev == X_dev || GV_dev == G_dev)) return HF_ERR_ARG;
  return hf::adjoint_impl(ctx, r, X_dev, ldx, G_dev, ldg, Lam_dev, ldl, GV_dev, static_cast<hipStream_t>(stream));
}

int hf_tune(hf_ctx* ctx, int32_t r, int32_t* front_min_host, int32_t* wide_min_host, double* ms_host,
            void* stream) {
  if (!ctx) return HF_ERR_ARG;
  return hf::tune_impl(ctx, r, front_min_host, wide_min_host, ms_host, static_cast<hipStream_t>(stream));
}

int hf_precond(hf_ctx* ctx, int32_t r, const double* R_dev, double* Y_dev, void* stream) {
  if (!ctx) return HF_ERR_ARG;
  return hf::precond_impl(ctx, r, R_dev, Y_dev, static_cast<hipStream_t>(stream));
}

int hf_kernel_dim(const hf_ctx* ctx, int32_t* k_host) {
  if (!ctx || !k_host) return HF_ERR_ARG;
  if (ctx->state < 2) return HF_ERR_STATE;
  *k_host = ctx->kdim;
  return HF_OK;
}

int hf_kernel_basis(const hf_ctx* ctx, double* N_dev, int64_t ldn, void* stream) {
  if (!ctx) return HF_ERR_ARG;
  return hf::kernel_basis_impl(ctx, N_dev, ldn, static_cast<hipStream_t>(stream));
}

int hf_schur(const hf_ctx* ctx, int32_t* m_host, int32_t* lambda2_host, double* S22_dev, int64_t lds,
             void* stream) {
  if (!ctx || !m_host) return HF_ERR_ARG;
  return hf::schur_impl(ctx, m_host, lambda2_host, S22_dev, lds, static_cast<hipStream_t>(stream));
}

int hf_scaling(const hf_ctx* ctx, double* q_dev, void* stream) {
  if (!ctx) return HF_ERR_ARG;
  return hf::scaling_impl(ctx, q_dev, static_cast<hipStream_t>(stream));
}

int hf_info(const hf_ctx* ctx, hf_info_t* info) {
  if (!ctx || !info) return HF_ERR_ARG;
  hf_info_t o{};
  o.n = ctx->n;
  o.nnz = ctx->nnz;
  o.n_nodes = ctx->n_nodes;
  o.n_levels = ctx->level_ptr.empty() ? 0 : (int32_t)ctx->level_ptr.size() - 1;
  o.max_front = ctx->max_front;
  o.max_pivots = ctx->max_p;
  o.factor_entries = ctx->factor_entries;
  o.factor_flops = ctx->flops_sym;
  o.factor_flops_done = ctx->flops_done;
  o.front_bytes = ctx->front_elems * (ctx->opt.low_precision == HF_PREC_FP64 ? 8 : 4);
  o.M = ctx->M;
  o.kernel_dim = ctx->kdim;
  o.gcr_blocks = ctx->gcr_blocks;
  o.gcr_iters_max = ctx->gcr_iters_max;
  o.gcr_iters_total = ctx->gcr_iters_total;
  o.solve_gcr_iters = ctx->solve_iters;
  o.rank_gap = ctx->rank_gap;
  o.rank_candidates = ctx->rank_candidates;
  o.state = ctx->state;
  o.t_analyse_ms = ctx->t_analyse;
  o.t_step1_ms = ctx->t_step1;
  o.t_gcr_ms = ctx->t_gcr;
  o.t_s22_ms = ctx->t_s22;
  o.t_solve_ms = ctx->t_solve;
  *info = o;
  return HF_OK;
}

int hf_pivots(const hf_ctx* ctx, int32_t* npiv_host, double* d_host, double* dstop_host, double* margin_host) {
  if (!ctx) return HF_ERR_ARG;
  if (ctx->state < 2) return HF_ERR_STATE;
  const int32_t nn = ctx->n_nodes;
  if ((int32_t)ctx->hstate.size() != nn) return HF_ERR_STATE;
  std::vector<double> d(ctx->n, 0.0);
  if ((d_host || margin_host) && ctx->n > 0) {
    if (ctx->factor_prec == HF_PREC_FP32) {
      std::vector<float> t(ctx->n);
      if (hipMemcpy(t.data(), ctx->d_dval.ptr, sizeof(float) * ctx->n, hipMemcpyDeviceToHost) != hipSuccess)
        return HF_ERR_HIP;
      for (int64_t i = 0; i < ctx->n; ++i) d[i] = t[i];
    } else if (hipMemcpy(d.data(), ctx->d_dval.ptr, sizeof(double) * ctx->n, hipMemcpyDeviceToHost) != hipSuccess) {
      return HF_ERR_HIP;
    }
  }
  const double tau = ctx->opt.tau;
  for (int32_t j = 0; j < nn; ++j) {
    const hf::NodeState& st = ctx->hstate[j];
    const int32_t s0 = ctx->nodes[j].start, p = ctx->nodes[j].p;
    for (int32_t k = st.npiv; k < p; ++k) d[s0 + k] = 0.0;  // postponed positions
    if (npiv_host) npiv_host[j] = st.npiv;
    if (dstop_host) dstop_host[j] = st.dstop;
    if (margin_host) {
      // the node's ratio tests: every accepted pivot against its reference, then
      // the candidate that stopped the node (a zero candidate is not a test)
      double m = INFINITY, ref = 1.0;
      bool have = ctx->opt.first_pivot_unit != 0;
      for (int32_t k = 0; k < st.npiv; ++k) {
        const double dk = d[s0 + k];
        if (have) m = std::min(m, std::fabs(std::log10(std::fabs(dk) / (tau * std::fabs(ref)))));
        ref = dk;
        have = true;
      }
      if (have && st.dstop == st.dstop && st.dstop != 0.0)
        m = std::min(m, std::fabs(std::log10(std::fabs(st.dstop) / (tau * std::fabs(ref)))));
      margin_host[j] = m;
    }
  }
  if (d_host) std::copy(d.begin(), d.end(), d_host);
  return HF_OK;
}

int hf_s22_pivots(const hf_ctx* ctx, double* mags_host) {
  if (!ctx || !mags_host) return HF_ERR_ARG;
  if (ctx->state < 2) return HF_ERR_STATE;
  if (ctx->M == 0) return HF_OK;
  if (hipMemcpy(mags_host, ctx->d_s22mag.ptr, sizeof(double) * ctx->M, hipMemcpyDeviceToHost) != hipSuccess)
    return HF_ERR_HIP;
  return HF_OK;
}

int hf_gcr_history(const hf_ctx* ctx, int32_t* nruns_host, int32_t* nfactor_host, int32_t* run_ptr_host,
                   double* hist_host) {
  if (!ctx || !nruns_host) return HF_ERR_ARG;
  const int32_t nr = (int32_t)ctx->hist_ptr.size() - 1;
  *nruns_host = nr;
  if (nfactor_host) *nfactor_host = ctx->hist_factor_runs;
  if (run_ptr_host) std::copy(ctx->hist_ptr.begin(), ctx->hist_ptr.end(), run_ptr_host);
  if (hist_host) std::copy(ctx->hist.begin(), ctx->hist.end(), hist_host);
  return HF_OK;
}

const char* hf_strerror(int status) {
  switch (status) {
    case HF_OK: return "ok";
    case HF_ERR_ARG: return "invalid argument";
    case HF_ERR_PATTERN: return "invalid sparsity pattern or ordering tree";
    case HF_ERR_VALUE: return "NaN or Inf among the matrix values";
    case HF_ERR_STATE: return "call out of order (analyse / factorize first)";
    case HF_ERR_NO_CONVERGENCE: return "block GCR did not converge";
    case HF_ERR_BREAKDOWN: return "block GCR breakdown";
    case HF_ERR_OOM: return "out of memory";
    case HF_ERR_HIP: return "HIP runtime error";
    case HF_ERR_NOT_IMPLEMENTED: return "not implemented for these sizes";
    default: return "unknown status";
  }
}

int hf_timing_enable(hf_ctx* ctx, int32_t on) {
  if (!ctx) return HF_ERR_ARG;
  ctx->timer.reset();
  ctx->timer.on = on != 0;
  return HF_OK;
}

int hf_timing_get(const hf_ctx* ctx, int32_t cls, hf_kstat_t* out) {
  if (!ctx || !out || cls < 0 || cls >= HF_K_NCLASS) return HF_ERR_ARG;
  out->ms = ctx->timer.ms[cls];
  out->launches = ctx->timer.n[cls];
  out->bytes = ctx->timer.bytes[cls];
  out->flops = ctx->timer.flops[cls];
  return HF_OK;
}

void hf_destroy(hf_ctx* ctx) { delete ctx; }

}  // extern "C"
