/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the variable-block sparse products of
 * the VBCSR paper.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does.  It shares no
 * code, header or table with the device library.
 *
 * Conventions (the readings documented with the library):
 *   - atom i carries b_i orbitals; off_0 = 0, off_{i+1} = off_i + b_i;
 *     a stored block (i, j) is a dense b_i x b_j matrix (section 2.1);
 *   - blocks are given in graph (CSR) order, each block row-major;
 *   - dense multi-vectors are row-major N x nrhs with a leading dimension.
 *
 * Everything is computed by expanding the blocks into scalar CSR and summing
 * every output element sequentially in FP64, in a fixed order, so the result
 * does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Scalar CSR expansion (block semantics of section 2.1).
 * Walk blocks k in graph order; block k of row i, column j = col_idx[k],
 * starting at value base_k, emits (off_i + p, off_j + q, v[base_k + p*b_j + q]).
 * Within a scalar row entries stay in block order, then ascending q.
 * Output arrays: rp[N+1], ci[nnz], va[nnz] (caller-allocated).            */
void oracle_expand(int32_t n, const int32_t *b, const int64_t *row_ptr,
                   const int32_t *col_idx, const double *vals,
                   int64_t *rp, int32_t *ci, double *va) {
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  off[0] = 0;
  for (int32_t i = 0; i < n; ++i) off[i + 1] = off[i] + b[i];
  int64_t N = off[n];
  /* count entries per scalar row */
  for (int64_t r = 0; r <= N; ++r) rp[r] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t width = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) width += b[col_idx[k]];
    for (int32_t p = 0; p < b[i]; ++p) rp[off[i] + p + 1] = width;
  }
  for (int64_t r = 0; r < N; ++r) rp[r + 1] += rp[r];
  /* fill, block row by block row (rows are independent) */
  int64_t *base_row = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  base_row[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t s = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += (int64_t)b[i] * b[col_idx[k]];
    base_row[i + 1] = base_row[i] + s;
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    int64_t base = base_row[i];
    int64_t fill = 0; /* position inside every scalar row of block row i */
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t j = col_idx[k];
      int32_t bj = b[j];
      for (int32_t p = 0; p < b[i]; ++p) {
        int64_t dst = rp[off[i] + p] + fill;
        for (int32_t q = 0; q < bj; ++q) {
          ci[dst + q] = (int32_t)(off[j] + q);
          va[dst + q] = vals[base + (int64_t)p * bj + q];
        }
      }
      base += (int64_t)b[i] * bj;
      fill += bj;
    }
  }
  free(base_row);
  free(off);
}

/* Y <- alpha * A * X + beta * Y on scalar CSR (forward product, section 3.2).
 * beta == 0 means Y is not read.  Each element is one sequential FP64 sum. */
void oracle_csr_spmm(int64_t N, const int64_t *rp, const int32_t *ci, const double *va,
                     const double *X, int64_t ldx, int32_t nrhs, double alpha, double beta,
                     double *Y, int64_t ldy) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < N; ++r) {
    for (int32_t c = 0; c < nrhs; ++c) {
      double acc = 0.0;
      for (int64_t e = rp[r]; e < rp[r + 1]; ++e) acc += va[e] * X[(int64_t)ci[e] * ldx + c];
      double y = alpha * acc;
      if (beta != 0.0) y += beta * Y[r * ldy + c];
      Y[r * ldy + c] = y;
    }
  }
}

/* Scalar transpose by a stable counting sort: entry (r, c, v) becomes (c, r, v);
 * inside a transposed row entries keep ascending source row order.  Applying
 * the forward product to it gives Y_j += sum_i A_ij^T X_i, the adjoint of
 * equation (1) for real data.  Output arrays: rpt[N+1], cit[nnz], vat[nnz]. */
void oracle_csr_transpose(int64_t N, const int64_t *rp, const int32_t *ci, const double *va,
                          int64_t *rpt, int32_t *cit, double *vat) {
  for (int64_t r = 0; r <= N; ++r) rpt[r] = 0;
  int64_t nnz = rp[N];
  for (int64_t e = 0; e < nnz; ++e) rpt[(int64_t)ci[e] + 1] += 1;
  for (int64_t r = 0; r < N; ++r) rpt[r + 1] += rpt[r];
  int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * ((size_t)N + 1));
  memcpy(cursor, rpt, sizeof(int64_t) * ((size_t)N + 1));
  for (int64_t r = 0; r < N; ++r) {
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
      int64_t dst = cursor[ci[e]]++;
      cit[dst] = (int32_t)r;
      vat[dst] = va[e];
    }
  }
  free(cursor);
}

/* Block-sampled product dA_k[p, q] = sum_c dY[off_i + p, c] * X[off_j + q, c]
 * for every stored block k = (i, j), written at base_k + p*b_j + q (graph
 * order, the layout of the input values).                                   */
void oracle_sddmm(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                  const double *dY, int64_t lddy, const double *X, int64_t ldx, int32_t nrhs,
                  double *dA) {
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t *base_row = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  off[0] = 0;
  base_row[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    off[i + 1] = off[i] + b[i];
    int64_t s = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += (int64_t)b[i] * b[col_idx[k]];
    base_row[i + 1] = base_row[i] + s;
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    int64_t base = base_row[i];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int32_t j = col_idx[k];
      for (int32_t p = 0; p < b[i]; ++p)
        for (int32_t q = 0; q < b[j]; ++q) {
          double acc = 0.0;
          for (int32_t c = 0; c < nrhs; ++c)
            acc += dY[(off[i] + p) * lddy + c] * X[(off[j] + q) * ldx + c];
          dA[base + (int64_t)p * b[j] + q] = acc;
        }
      base += (int64_t)b[i] * b[j];
    }
  }
  free(base_row);
  free(off);
}

/* Chebyshev moments of an already scaled operator (kernel polynomial method,
 * section 5):  T_0 = R, T_1 = A R, T_{k+1} = 2 A T_k - T_{k-1};
 * mu[k*nrhs + c] = sum_r R[r, c] * T_k[r, c] for k = 0..degree, each sum
 * taken sequentially over r.  Three N x nrhs work buffers are allocated here. */
int oracle_cheb(int64_t N, const int64_t *rp, const int32_t *ci, const double *va,
                const double *R, int64_t ldr, int32_t nrhs, int32_t degree, double *mu) {
  size_t sz = (size_t)N * (size_t)nrhs;
  double *t_prev = (double *)malloc(sizeof(double) * (sz ? sz : 1));
  double *t_cur = (double *)malloc(sizeof(double) * (sz ? sz : 1));
  if (!t_prev || !t_cur) { free(t_prev); free(t_cur); return -1; }
  for (int64_t r = 0; r < N; ++r)
    for (int32_t c = 0; c < nrhs; ++c) t_prev[r * nrhs + c] = R[r * ldr + c];
  for (int32_t k = 0; k <= degree; ++k) {
    if (k == 1) {
      oracle_csr_spmm(N, rp, ci, va, t_prev, nrhs, nrhs, 1.0, 0.0, t_cur, nrhs);
    } else if (k >= 2) {
      /* t_prev <- 2 A t_cur - t_prev, then swap the roles */
      oracle_csr_spmm(N, rp, ci, va, t_cur, nrhs, nrhs, 2.0, -1.0, t_prev, nrhs);
      double *tmp = t_prev; t_prev = t_cur; t_cur = tmp;
    }
    const double *tk = (k == 0) ? t_prev : t_cur;
    for (int32_t c = 0; c < nrhs; ++c) {
      double acc = 0.0;
      for (int64_t r = 0; r < N; ++r) acc += R[r * ldr + c] * tk[r * nrhs + c];
      mu[(int64_t)k * nrhs + c] = acc;
    }
  }
  free(t_prev);
  free(t_cur);
  return 0;
}

/* ------------------------------------------------------------------------
 * Thresholded block product C = A B (section 3.2, equations 2 and 3).
 * A and B are square operators over the same atoms (same b).
 * ---------------------------------------------------------------------- */

/* Frobenius norms of nblk blocks stored one after the other (block t has
 * size[t] values): the square root of the sum of the squares of its values,
 * summed in storage (row-major) order. */
void oracle_seq_norms(int64_t nblk, const int64_t *size, const double *vals, double *norms) {
  int64_t base = 0;
  for (int64_t t = 0; t < nblk; ++t) {
    double s = 0.0;
    for (int64_t e = 0; e < size[t]; ++e) s += vals[base + e] * vals[base + e];
    norms[t] = sqrt(s);
    base += size[t];
  }
}

/* Symbolic stage for the block rows rows[0..nrows).  For row i the candidate
 * columns are the columns j of every row k of B with a stored block (i, k)
 * in A; each candidate carries the bound of equation 3,
 *   U_ij = sum_k ||A_ik|| ||B_kj||,
 * summed over k in the order row i of A stores its blocks.  A candidate is
 * rejected when U_ij < eps.  The kept columns of each row are written in
 * ascending order to col[], their bounds to bound[], and cnt[t] receives
 * the number kept in row rows[t].  Returns the total, or -1 when it would
 * exceed cap.                                                              */
int64_t oracle_spgemm_symbolic(int32_t n, const int64_t *arp, const int32_t *aci,
                               const double *an, const int64_t *brp, const int32_t *bci,
                               const double *bn, double eps, const int64_t *rows,
                               int64_t nrows, int64_t *cnt, int32_t *col, double *bound,
                               int64_t cap) {
  double *acc = (double *)calloc((size_t)n + 1, sizeof(double));
  char *seen = (char *)calloc((size_t)n + 1, 1);
  int64_t total = 0;
  for (int64_t t = 0; t < nrows; ++t) {
    int64_t i = rows[t];
    for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
      int32_t k = aci[ka];
      for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
        int32_t j = bci[kb];
        seen[j] = 1;
        acc[j] += an[ka] * bn[kb];
      }
    }
    /* ascending scan of the atom range keeps the columns sorted */
    int64_t kept = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (!seen[j]) continue;
      if (!(acc[j] < eps)) {
        if (total + kept >= cap) { free(acc); free(seen); return -1; }
        col[total + kept] = j;
        bound[total + kept] = acc[j];
        ++kept;
      }
      seen[j] = 0;
      acc[j] = 0.0;
    }
    cnt[t] = kept;
    total += kept;
  }
  free(acc);
  free(seen);
  return total;
}

/* Numeric stage: the blocks C_ij = sum_k A_ik B_kj (equation 2) of a given
 * pattern, for the block rows rows[0..nrows) whose kept columns are
 * col[crp[t] .. crp[t+1]) (ascending).  Element (p, q) of C_ij is one
 * sequential FP64 sum over k in the order row i of A stores its blocks, then
 * over the inner index ascending.  Blocks are written row-major, one after
 * the other in pattern order, to out[].                                     */
void oracle_spgemm_numeric(int32_t n, const int32_t *b, const int64_t *arp, const int32_t *aci,
                           const double *av, const int64_t *brp, const int32_t *bci,
                           const double *bv, const int64_t *rows, int64_t nrows,
                           const int64_t *crp, const int32_t *col, double *out) {
  int64_t *abase = (int64_t *)malloc(sizeof(int64_t) * ((size_t)arp[n] + 1));
  int64_t *bbase = (int64_t *)malloc(sizeof(int64_t) * ((size_t)brp[n] + 1));
  int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  abase[0] = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = arp[i]; k < arp[i + 1]; ++k)
      abase[k + 1] = abase[k] + (int64_t)b[i] * b[aci[k]];
  bbase[0] = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = brp[i]; k < brp[i + 1]; ++k)
      bbase[k + 1] = bbase[k] + (int64_t)b[i] * b[bci[k]];
  for (int32_t j = 0; j < n; ++j) slot[j] = -1;
  int64_t obase = 0;
  for (int64_t t = 0; t < nrows; ++t) {
    int64_t i = rows[t];
    int32_t bi = b[i];
    /* output position of every kept column of this row */
    for (int64_t c = crp[t]; c < crp[t + 1]; ++c) {
      slot[col[c]] = obase;
      int64_t sz = (int64_t)bi * b[col[c]];
      for (int64_t e = 0; e < sz; ++e) out[obase + e] = 0.0;
      obase += sz;
    }
    for (int64_t ka = arp[i]; ka < arp[i + 1]; ++ka) {
      int32_t k = aci[ka];
      int32_t bk = b[k];
      const double *A = av + abase[ka];
      for (int64_t kb = brp[k]; kb < brp[k + 1]; ++kb) {
        int32_t j = bci[kb];
        if (slot[j] < 0) continue;
        int32_t bj = b[j];
        const double *B = bv + bbase[kb];
        double *C = out + slot[j];
        for (int32_t p = 0; p < bi; ++p)
          for (int32_t q = 0; q < bj; ++q)
            for (int32_t s = 0; s < bk; ++s) C[p * bj + q] += A[p * bk + s] * B[s * bj + q];
      }
    }
    for (int64_t c = crp[t]; c < crp[t + 1]; ++c) slot[col[c]] = -1;
  }
  free(slot);
  free(bbase);
  free(abase);
}
