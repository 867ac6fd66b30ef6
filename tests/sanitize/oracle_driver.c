/* Sanitizer driver for the CPU oracle -- test infrastructure, built with gcc
 * -fsanitize=address,undefined by tests/test_sanitizers.py.  It runs every
 * oracle routine on a random block graph and a dense multi-vector. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_expand(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                   const double *vals, int64_t *rp, int32_t *ci, double *va);
void oracle_csr_spmm(int64_t N, const int64_t *rp, const int32_t *ci, const double *va,
                     const double *X, int64_t ldx, int32_t nrhs, double alpha, double beta,
                     double *Y, int64_t ldy);
void oracle_csr_transpose(int64_t N, const int64_t *rp, const int32_t *ci, const double *va,
                          int64_t *rpt, int32_t *cit, double *vat);
void oracle_sddmm(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                  const double *dY, int64_t lddy, const double *X, int64_t ldx, int32_t nrhs,
                  double *dA);
int oracle_cheb(int64_t N, const int64_t *rp, const int32_t *ci, const double *va, const double *R,
                int64_t ldr, int32_t nrhs, int32_t degree, double *mu);
void oracle_seq_norms(int64_t nblk, const int64_t *size, const double *vals, double *norms);
int64_t oracle_spgemm_symbolic(int32_t n, const int64_t *arp, const int32_t *aci, const double *an,
                               const int64_t *brp, const int32_t *bci, const double *bn,
                               double eps, const int64_t *rows, int64_t nrows, int64_t *cnt,
                               int32_t *col, double *bound, int64_t cap);
void oracle_spgemm_numeric(int32_t n, const int32_t *b, const int64_t *arp, const int32_t *aci,
                           const double *av, const int64_t *brp, const int32_t *bci,
                           const double *bv, const int64_t *rows, int64_t nrows,
                           const int64_t *crp, const int32_t *col, double *out);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}

int main(void) {
  const int32_t n = 400, nrhs = 5;
  int32_t *b = malloc(sizeof(int32_t) * n);
  int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
  int32_t *ci = malloc(sizeof(int32_t) * n * 12);
  int64_t nnzb = 0, nval = 0, N = 0;
  for (int32_t i = 0; i < n; ++i) b[i] = 1 + (int32_t)(rnd() % 9), N += b[i];
  rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    char used[400] = {0};
    int d = (int)(rnd() % 12);
    for (int t = 0; t < d; ++t) {
      int32_t j = (int32_t)(rnd() % n);
      if (used[j]) continue;
      used[j] = 1;
      ci[nnzb++] = j;
      nval += (int64_t)b[i] * b[j];
    }
    rp[i + 1] = nnzb;
  }
  double *v = malloc(sizeof(double) * (nval ? nval : 1));
  for (int64_t e = 0; e < nval; ++e) v[e] = (double)(rnd() % 2001) / 1000.0 - 1.0;
  int64_t *srp = malloc(sizeof(int64_t) * (N + 1)), *trp = malloc(sizeof(int64_t) * (N + 1));
  int32_t *sci = malloc(sizeof(int32_t) * (nval ? nval : 1)), *tci = malloc(sizeof(int32_t) * (nval ? nval : 1));
  double *sva = malloc(sizeof(double) * (nval ? nval : 1)), *tva = malloc(sizeof(double) * (nval ? nval : 1));
  oracle_expand(n, b, rp, ci, v, srp, sci, sva);
  oracle_csr_transpose(N, srp, sci, sva, trp, tci, tva);
  double *X = malloc(sizeof(double) * N * nrhs), *Y = malloc(sizeof(double) * N * nrhs);
  for (int64_t e = 0; e < N * nrhs; ++e) X[e] = (double)(rnd() % 2001) / 1000.0 - 1.0, Y[e] = 0.5;
  oracle_csr_spmm(N, srp, sci, sva, X, nrhs, nrhs, 1.0, 0.5, Y, nrhs);
  oracle_csr_spmm(N, trp, tci, tva, X, nrhs, nrhs, 2.0, 0.0, Y, nrhs);
  double *dA = malloc(sizeof(double) * (nval ? nval : 1));
  oracle_sddmm(n, b, rp, ci, X, nrhs, Y, nrhs, nrhs, dA);
  double *mu = malloc(sizeof(double) * 17 * nrhs);
  int rc = oracle_cheb(N, srp, sci, sva, X, nrhs, nrhs, 16, mu);
  int64_t *sizes = malloc(sizeof(int64_t) * (nnzb ? nnzb : 1));
  for (int32_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) sizes[k] = (int64_t)b[i] * b[ci[k]];
  double *nrm = malloc(sizeof(double) * (nnzb ? nnzb : 1));
  oracle_seq_norms(nnzb, sizes, v, nrm);
  int64_t *rows = malloc(sizeof(int64_t) * n), *cnt = malloc(sizeof(int64_t) * n);
  for (int32_t i = 0; i < n; ++i) rows[i] = i;
  int64_t cap = nnzb * 12 + 1;
  int32_t *col = malloc(sizeof(int32_t) * cap);
  double *bound = malloc(sizeof(double) * cap);
  int64_t tot = oracle_spgemm_symbolic(n, rp, ci, nrm, rp, ci, nrm, 0.5, rows, n, cnt, col, bound, cap);
  int64_t *crp = malloc(sizeof(int64_t) * (n + 1));
  crp[0] = 0;
  int64_t cvals = 0;
  for (int32_t i = 0; i < n; ++i) crp[i + 1] = crp[i] + cnt[i];
  for (int32_t i = 0; i < n; ++i)
    for (int64_t t = crp[i]; t < crp[i + 1]; ++t) cvals += (int64_t)b[i] * b[col[t]];
  double *cv = malloc(sizeof(double) * (cvals ? cvals : 1));
  oracle_spgemm_numeric(n, b, rp, ci, v, rp, ci, v, rows, n, crp, col, cv);
  double chk = 0.0;
  for (int64_t e = 0; e < N * nrhs; ++e) chk += Y[e];
  printf("oracle driver: rc %d, %lld products kept, checksum %.6f\n", rc, (long long)tot,
         chk + mu[0] + (cvals ? cv[0] : 0.0) + (nval ? dA[0] : 0.0));
  free(b); free(rp); free(ci); free(v); free(srp); free(trp); free(sci); free(tci); free(sva);
  free(tva); free(X); free(Y); free(dA); free(mu); free(sizes); free(nrm); free(rows); free(cnt);
  free(col); free(bound); free(crp); free(cv);
  return rc != 0 || tot < 0;
}
