/*
 * ORACLE (test infrastructure only; never part of the product path).
 *
 * Plain CPU implementation of step 1 of the hybrid factorization (Algorithm 1,
 * step 1, Sec. 3) and of the preconditioner application built on it
 * (Sec. 3.1-3.3).  This file is compiled twice, with REAL = float and with
 * REAL = double, giving the low-precision and the FP64 variant.
 *
 * Step 1 follows Sec. 2.1-2.2 literally, organised along the elimination tree
 * of the nested-dissection ordering (one dense frontal matrix per tree node):
 *   - the front of node j holds its own indices Lambda_j followed by its border
 *     (ancestor indices coupled to the subtree); entries of K are assigned, the
 *     children's Schur-complement blocks are added (extend-add);
 *   - pivots are searched among the remaining diagonal entries of Lambda_j only:
 *     the entry of largest magnitude is moved to the front by a symmetric
 *     exchange and eliminated by the rank-1 update with weight 1/d of eq. (2);
 *     ties go to the smallest global (nested-dissection) index;
 *   - threshold postponing (Sec. 2.2): when |d_next / d_prev| < tau the rest of
 *     Lambda_j is not factorized.  The first pivot of a node is compared with 1
 *     (the unit diagonal produced by the scaling of Sec. 2) unless
 *     first_ref_unit == 0, in which case it is always accepted (if nonzero);
 *     a zero pivot is always postponed;
 *   - postponed indices are removed from the low-precision factorization: they
 *     are never eliminated and are not passed to the parent.
 * Only the lower triangle of each front is kept.  No blocking: one rank-1
 * update per pivot, as in eq. (2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#error "compile with -DREAL=float or -DREAL=double and -DSUFFIX=..."
#endif

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SUFFIX)

#define AT(F, ld, r, c) (F)[(size_t)(c) * (size_t)(ld) + (size_t)(r)]

/* symmetric exchange of positions i < k in a lower-triangular col-major front */
static void FN(sym_swap)(REAL* F, int64_t f, int64_t i, int64_t k) {
  REAL t;
  if (i == k) return;
  for (int64_t c = 0; c < i; ++c) { t = AT(F, f, i, c); AT(F, f, i, c) = AT(F, f, k, c); AT(F, f, k, c) = t; }
  t = AT(F, f, i, i); AT(F, f, i, i) = AT(F, f, k, k); AT(F, f, k, k) = t;
  for (int64_t c = i + 1; c < k; ++c) { t = AT(F, f, c, i); AT(F, f, c, i) = AT(F, f, k, c); AT(F, f, k, c) = t; }
  for (int64_t r = k + 1; r < f; ++r) { t = AT(F, f, r, i); AT(F, f, r, i) = AT(F, f, r, k); AT(F, f, r, k) = t; }
}

/*
 * Multifrontal partial LDL^T with postponing.
 *   n, indptr, indices, vals : scaled matrix K in the elimination (permuted)
 *                              order, full symmetric CSR, FP64 values.
 *   node_ptr, parent         : the nested-dissection tree, postorder.
 *   border_ptr, border       : border index lists (sorted) of every node.
 *   lptr                     : offsets of the per-node panels in Lstore
 *                              (node j: (p_j + b_j) x p_j, column-major).
 * Outputs:
 *   Lstore  : per node, rows in front order [accepted pivots, postponed, border],
 *             columns 0..npiv-1 hold the unit-lower factor L (diagonal not stored
 *             meaningfully);
 *   dstore  : D of the accepted pivots, at position node_ptr[j] + k;
 *   piv_order[node_ptr[j] + k] : global index eliminated k-th (k < npiv[j]) or
 *             postponed (k >= npiv[j]);
 *   npiv    : number of accepted pivots per node;
 *   margin  : per node, min |log10(|d_k0| / (tau |d_prev|))| over its tests
 *             (+inf when no test was made);
 *   dstop   : per node, the diagonal value of the candidate that stopped the
 *             node (NaN when every candidate was accepted);
 *   tiegap  : per node, min over its accepted pivots of (|d| - r) / |d|, r the
 *             largest |diagonal| among the other candidates of that selection,
 *             over the selections where the winner or that rival is a computed
 *             value (changed by an extend-add or an elimination; two untouched
 *             entries of K tie identically in any arithmetic); +inf when no
 *             such selection had a rival.
 *   exclude : optional mask over global indices; masked indices are never
 *             pivot candidates and end up with the postponed ones (used to build
 *             a factorization of K11 for a given split).
 * Returns 0, or -1 when an entry falls outside the front (ordering is not a
 * valid nested dissection), -2 on allocation failure.
 */
int FN(hfo_factor_)(int64_t n, const int64_t* indptr, const int32_t* indices, const double* vals,
                    int32_t n_nodes, const int32_t* node_ptr, const int32_t* parent,
                    const int64_t* border_ptr, const int32_t* border, double tau,
                    int32_t first_ref_unit, const uint8_t* exclude, const int64_t* lptr,
                    REAL* Lstore, REAL* dstore, int32_t* piv_order, int32_t* npiv,
                    double* margin, double* dstop, double* tiegap) {
  int rc = 0;
  int32_t* loc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  REAL** contrib = (REAL**)calloc((size_t)(n_nodes > 0 ? n_nodes : 1), sizeof(REAL*));
  /* children lists */
  int32_t* nchild = (int32_t*)calloc((size_t)n_nodes + 1, sizeof(int32_t));
  int32_t* cptr = (int32_t*)calloc((size_t)n_nodes + 1, sizeof(int32_t));
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
  if (!loc || !contrib || !nchild || !cptr || !clist) { rc = -2; goto done; }
  for (int64_t g = 0; g < n; ++g) loc[g] = -1;
  for (int32_t j = 0; j < n_nodes; ++j) if (parent[j] >= 0) nchild[parent[j]]++;
  for (int32_t j = 0; j < n_nodes; ++j) cptr[j + 1] = cptr[j] + nchild[j];
  memset(nchild, 0, sizeof(int32_t) * (size_t)n_nodes);
  for (int32_t j = 0; j < n_nodes; ++j)
    if (parent[j] >= 0) { int32_t pj = parent[j]; clist[cptr[pj] + nchild[pj]++] = j; }

  for (int32_t j = 0; j < n_nodes; ++j) {
    const int64_t s = node_ptr[j], p = node_ptr[j + 1] - node_ptr[j];
    const int64_t b = border_ptr[j + 1] - border_ptr[j], f = p + b;
    const int32_t* bj = border + border_ptr[j];
    REAL* F = (REAL*)calloc((size_t)(f * f > 0 ? f * f : 1), sizeof(REAL));
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(f > 0 ? f : 1));
    REAL* w = (REAL*)malloc(sizeof(REAL) * (size_t)(f > 0 ? f : 1));
    uint8_t* tch = (uint8_t*)calloc((size_t)(f > 0 ? f : 1), 1);   /* diagonal is a computed value */
    if (!F || !idx || !w || !tch) { free(F); free(idx); free(w); free(tch); rc = -2; goto done; }
    for (int64_t k = 0; k < p; ++k) { loc[s + k] = (int32_t)k; idx[k] = (int32_t)(s + k); }
    for (int64_t k = 0; k < b; ++k) { loc[bj[k]] = (int32_t)(p + k); idx[p + k] = bj[k]; }

    /* assemble the entries of K owned by this node */
    for (int64_t k = 0; k < p; ++k) {
      const int64_t g = s + k;
      for (int64_t e = indptr[g]; e < indptr[g + 1]; ++e) {
        const int64_t c = indices[e];
        if (c < s) continue;                 /* assembled in a descendant front */
        const int32_t lc = loc[c];
        if (lc < 0) { free(F); free(idx); free(w); free(tch); rc = -1; goto done; }
        const int64_t r0 = lc > k ? lc : k, c0 = lc > k ? k : lc;
        AT(F, f, r0, c0) = (REAL)vals[e];
      }
    }
    /* extend-add of the children's Schur-complement blocks */
    for (int32_t ci = cptr[j]; ci < cptr[j + 1]; ++ci) {
      const int32_t c = clist[ci];
      const int64_t bc = border_ptr[c + 1] - border_ptr[c];
      const int32_t* bcl = border + border_ptr[c];
      REAL* C = contrib[c];
      for (int64_t t = 0; t < bc; ++t) {
        const int32_t lt = loc[bcl[t]];
        for (int64_t r = t; r < bc; ++r) {
          const int32_t lr = loc[bcl[r]];
          if (lr < 0 || lt < 0) { free(F); free(idx); free(w); free(tch); rc = -1; goto done; }
          const int32_t r0 = lr > lt ? lr : lt, c0 = lr > lt ? lt : lr;
          AT(F, f, r0, c0) += AT(C, bc, r, t);
          if (r0 == c0) tch[r0] = 1;
        }
      }
      free(C);
      contrib[c] = NULL;
    }

    /* partial factorization of the pivot block with postponing */
    double dprev = 1.0;
    int have_prev = first_ref_unit ? 1 : 0;
    double mmin = INFINITY;
    double stopv = NAN;
    double gmin = INFINITY;
    int64_t i;
    for (i = 0; i < p; ++i) {
      int64_t k0 = -1;
      double best = -1.0;
      for (int64_t k = i; k < p; ++k) {
        if (exclude && exclude[idx[k]]) continue;
        const double v = fabs((double)AT(F, f, k, k));
        if (v > best || (v == best && idx[k] < idx[k0])) { best = v; k0 = k; }
      }
      double rival = -1.0;                   /* largest rival that can tie in another arithmetic */
      for (int64_t k = i; k < p && k0 >= 0; ++k) {
        if (k == k0 || (exclude && exclude[idx[k]])) continue;
        if (!tch[k] && !tch[k0]) continue;
        const double v = fabs((double)AT(F, f, k, k));
        if (v > rival) rival = v;
      }
      if (k0 < 0) break;                     /* only excluded indices remain */
      const double dk = (double)AT(F, f, k0, k0);
      if (dk == 0.0) { stopv = 0.0; break; }
      if (have_prev) {
        const double ratio = fabs(dk) / (tau * fabs(dprev));
        const double m = fabs(log10(ratio));
        if (m < mmin) mmin = m;
        if (fabs(dk) < tau * fabs(dprev)) { stopv = dk; break; }
      }
      if (rival >= 0.0 && (best - rival) / best < gmin) gmin = (best - rival) / best;
      FN(sym_swap)(F, f, i, k0);
      { int32_t t = idx[i]; idx[i] = idx[k0]; idx[k0] = t; }
      { uint8_t t = tch[i]; tch[i] = tch[k0]; tch[k0] = t; }
      for (int64_t r = i + 1; r < p; ++r) if (AT(F, f, r, i) != (REAL)0) tch[r] = 1;
      const REAL d = AT(F, f, i, i);
      for (int64_t r = i + 1; r < f; ++r) w[r] = AT(F, f, r, i);
      /* eq. (2): S' = K'_22 - col d^{-1} row, lower triangle only */
#pragma omp parallel for schedule(static) if (f - i > 384)
      for (int64_t c = i + 1; c < f; ++c) {
        const REAL wc = w[c] / d;
        REAL* Fc = &AT(F, f, 0, c);
        for (int64_t r = c; r < f; ++r) Fc[r] -= w[r] * wc;
      }
      for (int64_t r = i + 1; r < f; ++r) AT(F, f, r, i) = w[r] / d;
      dstore[s + i] = d;
      dprev = (double)d;
      have_prev = 1;
    }
    npiv[j] = (int32_t)i;
    margin[j] = mmin;
    dstop[j] = stopv;
    tiegap[j] = gmin;
    for (int64_t k = 0; k < p; ++k) piv_order[s + k] = idx[k];
    /* the panel (all rows, p columns) goes to the factor store */
    memcpy(Lstore + lptr[j], F, sizeof(REAL) * (size_t)(f * p));
    /* Schur-complement block of the border for the parent (postponed rows dropped) */
    if (b > 0 && parent[j] >= 0) {
      REAL* C = (REAL*)malloc(sizeof(REAL) * (size_t)(b * b));
      if (!C) { free(F); free(idx); free(w); free(tch); rc = -2; goto done; }
      for (int64_t c = 0; c < b; ++c)
        for (int64_t r = 0; r < b; ++r) AT(C, b, r, c) = AT(F, f, p + r, p + c);
      contrib[j] = C;
    }
    for (int64_t k = 0; k < f; ++k) loc[idx[k]] = -1;
    free(F); free(idx); free(w); free(tch);
  }
done:
  if (contrib) for (int32_t j = 0; j < n_nodes; ++j) free(contrib[j]);
  free(contrib); free(loc); free(nchild); free(cptr); free(clist);
  return rc;
}

/*
 * Preconditioner Q^{-1} of Sec. 3.2: for each FP64 column r (elimination order),
 * cast to REAL (round to nearest), forward substitution with L over the tree in
 * postorder, division by D, backward substitution with L^T, cast back.  Indices
 * of the hard part (is_l2[g] != 0) are excluded: they are set to zero before the
 * backward sweep and in the result.
 *   R, Y : column-major n x nrhs, leading dimension n.
 */
void FN(hfo_precond_)(int64_t n, int32_t n_nodes, const int32_t* node_ptr, const int64_t* border_ptr,
                      const int32_t* border, const int64_t* lptr, const REAL* Lstore,
                      const REAL* dstore, const int32_t* piv_order, const int32_t* npiv,
                      const uint8_t* is_l2, int32_t nrhs, const double* R, double* Y) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t col = 0; col < nrhs; ++col) {
    REAL* y = (REAL*)malloc(sizeof(REAL) * (size_t)(n > 0 ? n : 1));
    for (int64_t g = 0; g < n; ++g) y[g] = is_l2[g] ? (REAL)0 : (REAL)R[(size_t)col * n + g];
    /* forward: L z = y */
    for (int32_t j = 0; j < n_nodes; ++j) {
      const int64_t s = node_ptr[j], p = node_ptr[j + 1] - node_ptr[j];
      const int64_t b = border_ptr[j + 1] - border_ptr[j], f = p + b;
      const int32_t* bj = border + border_ptr[j];
      const REAL* L = Lstore + lptr[j];
      for (int64_t k = 0; k < npiv[j]; ++k) {
        const REAL z = y[piv_order[s + k]];
        for (int64_t r = k + 1; r < f; ++r) {
          const int64_t g = r < p ? piv_order[s + r] : bj[r - p];
          y[g] -= AT(L, f, r, k) * z;
        }
      }
    }
    /* D^{-1} on the accepted pivots; the hard part is excluded */
    for (int32_t j = 0; j < n_nodes; ++j) {
      const int64_t s = node_ptr[j];
      for (int64_t k = 0; k < npiv[j]; ++k) y[piv_order[s + k]] /= dstore[s + k];
    }
    for (int64_t g = 0; g < n; ++g) if (is_l2[g]) y[g] = (REAL)0;
    /* backward: L^T x = y */
    for (int32_t j = n_nodes - 1; j >= 0; --j) {
      const int64_t s = node_ptr[j], p = node_ptr[j + 1] - node_ptr[j];
      const int64_t b = border_ptr[j + 1] - border_ptr[j], f = p + b;
      const int32_t* bj = border + border_ptr[j];
      const REAL* L = Lstore + lptr[j];
      for (int64_t k = npiv[j] - 1; k >= 0; --k) {
        REAL acc = y[piv_order[s + k]];
        for (int64_t r = k + 1; r < f; ++r) {
          const int64_t g = r < p ? piv_order[s + r] : bj[r - p];
          acc -= AT(L, f, r, k) * y[g];
        }
        y[piv_order[s + k]] = acc;
      }
    }
    for (int64_t g = 0; g < n; ++g) Y[(size_t)col * n + g] = is_l2[g] ? 0.0 : (double)y[g];
    free(y);
  }
}
