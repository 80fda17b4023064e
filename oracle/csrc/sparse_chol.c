/*
 * Plain sparse Cholesky factorisation A = L L^T of a symmetric positive
 * definite matrix, for the CPU oracle (test infrastructure only).
 *
 * The caller passes the matrix already symmetrically permuted (a fill
 * reducing order is chosen in Python) as a full symmetric pattern in
 * compressed-column form. Steps, all textbook:
 *   1. elimination tree: parent(j) = min{ i > j : L(i, j) != 0 }, found
 *      column by column by walking from each i < j with A(i, j) != 0 up its
 *      current root path (with path compression);
 *   2. column structures: rows of L(:, j) below the diagonal are the rows
 *      i > j of A(:, j) together with the structures of j's children in the
 *      tree, minus j itself;
 *   3. left-looking numeric factorisation: column j of L is A(j:n, j) minus
 *      L(j:n, k) L(j, k) for every earlier column k with L(j, k) != 0, then
 *      divided by the square root of its diagonal. The columns k with a
 *      non-zero in row j are kept in linked lists keyed by the next row each
 *      column still has to contribute to.
 * Solves run forward substitution with L and back substitution with L^T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int n;
  int64_t *Lp; /* n+1 column starts; first entry of each column is the diagonal */
  int *Li;     /* row indices, ascending within a column */
  double *Lx;
} chol_t;

static int cmp_int(const void *a, const void *b) {
  const int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

void chol_free(void *h) {
  chol_t *c = (chol_t *)h;
  if (!c) return;
  free(c->Lp);
  free(c->Li);
  free(c->Lx);
  free(c);
}

int64_t chol_nnz(void *h) { return h ? ((chol_t *)h)->Lp[((chol_t *)h)->n] : 0; }

/* Returns 0 on success, 1 if the matrix is not positive definite, 2 on
 * allocation failure. Ap/Ai/Ax: full symmetric pattern, compressed columns. */
int chol_factor(int n, const int64_t *Ap, const int *Ai, const double *Ax, void **out) {
  *out = NULL;
  int *parent = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *anc = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  if (!parent || !anc) return 2;
  /* 1. elimination tree */
  for (int j = 0; j < n; ++j) {
    parent[j] = -1;
    anc[j] = -1;
    for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
      int i = Ai[p];
      while (i != -1 && i < j) {
        const int next = anc[i];
        anc[i] = j; /* path compression towards j */
        if (next == -1) parent[i] = j;
        i = next;
      }
    }
  }
  free(anc);
  /* children lists */
  int *child_head = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *child_next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *mark = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *tmp = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int64_t *Lp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!child_head || !child_next || !mark || !tmp || !Lp) return 2;
  for (int j = 0; j < n; ++j) child_head[j] = -1, mark[j] = -1;
  for (int j = n - 1; j >= 0; --j) {
    if (parent[j] >= 0) {
      child_next[j] = child_head[parent[j]];
      child_head[parent[j]] = j;
    }
  }
  /* 2. column structures (diagonal first, then rows > j ascending) */
  int64_t cap = 8 * (int64_t)n + 16, used = 0;
  int *Li = (int *)malloc(sizeof(int) * (size_t)cap);
  if (!Li) return 2;
  for (int j = 0; j < n; ++j) {
    int cnt = 0;
    Lp[j] = used; /* also ends column j-1, whose structure children read below */
    mark[j] = j;
    for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
      const int i = Ai[p];
      if (i > j && mark[i] != j) { mark[i] = j; tmp[cnt++] = i; }
    }
    for (int c = child_head[j]; c != -1; c = child_next[c]) {
      for (int64_t p = Lp[c] + 1; p < Lp[c + 1]; ++p) {
        const int i = Li[p];
        if (i > j && mark[i] != j) { mark[i] = j; tmp[cnt++] = i; }
      }
    }
    qsort(tmp, (size_t)cnt, sizeof(int), cmp_int);
    if (used + cnt + 1 > cap) {
      while (used + cnt + 1 > cap) cap *= 2;
      int *nl = (int *)realloc(Li, sizeof(int) * (size_t)cap);
      if (!nl) return 2;
      Li = nl;
    }
    Li[used++] = j;
    memcpy(Li + used, tmp, sizeof(int) * (size_t)cnt);
    used += cnt;
  }
  Lp[n] = used;
  free(child_head);
  free(child_next);
  free(parent);
  free(mark);
  free(tmp);
  /* 3. numeric, left-looking */
  double *Lx = (double *)malloc(sizeof(double) * (size_t)(used > 0 ? used : 1));
  double *x = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  int64_t *nextpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int *head = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *link = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  if (!Lx || !x || !nextpos || !head || !link) return 2;
  for (int j = 0; j < n; ++j) head[j] = -1;
  int status = 0;
  for (int j = 0; j < n && status == 0; ++j) {
    for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p)
      if (Ai[p] >= j) x[Ai[p]] = Ax[p];
    int k = head[j];
    head[j] = -1;
    while (k != -1) {
      const int knext = link[k];
      const int64_t pos = nextpos[k]; /* entry of row j in column k */
      const double ljk = Lx[pos];
      for (int64_t p = pos; p < Lp[k + 1]; ++p) x[Li[p]] -= Lx[p] * ljk;
      nextpos[k] = pos + 1;
      if (pos + 1 < Lp[k + 1]) {
        const int r = Li[pos + 1];
        link[k] = head[r];
        head[r] = k;
      }
      k = knext;
    }
    const double d = x[j];
    if (!(d > 0.0)) { status = 1; break; }
    const double ljj = sqrt(d);
    Lx[Lp[j]] = ljj;
    x[j] = 0.0;
    for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
      Lx[p] = x[Li[p]] / ljj;
      x[Li[p]] = 0.0;
    }
    nextpos[j] = Lp[j] + 1;
    if (Lp[j] + 1 < Lp[j + 1]) {
      const int r = Li[Lp[j] + 1];
      link[j] = head[r];
      head[r] = j;
    }
  }
  free(x);
  free(nextpos);
  free(head);
  free(link);
  if (status) {
    free(Lp);
    free(Li);
    free(Lx);
    return status;
  }
  chol_t *c = (chol_t *)malloc(sizeof(chol_t));
  if (!c) return 2;
  c->n = n;
  c->Lp = Lp;
  c->Li = Li;
  c->Lx = Lx;
  *out = c;
  return 0;
}

/* Solves L L^T x = b in place for nrhs right-hand sides stored one after
 * the other (each of length n). */
void chol_solve(void *h, double *b, int nrhs) {
  const chol_t *c = (const chol_t *)h;
  const int n = c->n;
  for (int r = 0; r < nrhs; ++r) {
    double *y = b + (int64_t)r * n;
    for (int j = 0; j < n; ++j) { /* L y = b */
      const double yj = y[j] / c->Lx[c->Lp[j]];
      y[j] = yj;
      for (int64_t p = c->Lp[j] + 1; p < c->Lp[j + 1]; ++p) y[c->Li[p]] -= c->Lx[p] * yj;
    }
    for (int j = n - 1; j >= 0; --j) { /* L^T x = y */
      double s = y[j];
      for (int64_t p = c->Lp[j] + 1; p < c->Lp[j + 1]; ++p) s -= c->Lx[p] * y[c->Li[p]];
      y[j] = s / c->Lx[c->Lp[j]];
    }
  }
}
